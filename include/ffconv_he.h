/*
 * ffconv_he.h -- C ABI of the MI355X (gfx950) homomorphic convolution library.
 *
 * The library evaluates convolution layers on packed RLWE ciphertexts of an
 * RNS CKKS-style scheme, in the two forms of the FFConv paper (arXiv
 * 2102.03494): a plain d x d convolution under DensePack (Section 3.2,
 * Fig. 1, Table I) and the FFConv factorisation (Section 4, Eq. 2): a
 * low-rank d x d convolution under DensePack, the DP->CP transition
 * (Table III, d = 1) and a 1 x 1 convolution under ConvPack (Table II).
 * The setting is the paper's (Section 1 and Section 3): the client encrypts
 * an image, the server holds plaintext weights and returns an encrypted
 * prediction.  Every step runs in hand-written HIP kernels.
 *
 * Conventions shared by all calls
 * -------------------------------
 * Ring: Z[X]/(X^N + 1), N a power of two in [2^10, 2^14].  Moduli: the
 * ciphertext primes q_0 > ... > q_{L-1} (ordered as generated) followed by the
 * special prime P; "modulus index" t < L means q_t and t = L means P.  Every
 * prime is 1 mod 2N and below 2^62.
 *
 * Polynomials are stored limb-major as uint64 residues in [0, q):
 *   poly  = [n_limbs][N], limb t reduced mod modulus index t;
 *   ct    = [2][level][N]   (c0 then c1; decryption is c0 + c1*s);
 *   batch = [count][2][level][N], contiguous.
 * Ciphertexts and plaintexts are in the NTT domain: entry i holds the value
 * at psi^(2*brv(i)+1), with psi = x^((q-1)/2N) for x the smallest quadratic
 * non-residue mod q and brv the log2(N)-bit reversal.  Slot j of a CKKS
 * vector is the evaluation at zeta^(5^j), zeta = exp(i pi / N); the Galois
 * element 5^k mod 2N rotates the slot vector left by k.
 *
 * Memory: every data pointer named d_* is device memory owned by the caller
 * (e.g. torch tensors).  Host pointers are named h_*.  The library owns the
 * context tables and the switching keys (he_keys_upload copies client-made
 * keys into it).  The workspace arena that evaluation calls take their
 * temporaries from is either the caller's (he_ctx_set_workspace) or the
 * library's (he_ctx_reserve).  Only he_ctx_create, he_ctx_reserve,
 * he_keys_upload and the client helper he_keygen_switch allocate device
 * memory; evaluation calls never do (a call that needs more workspace than
 * there is returns HE_ENOMEM).
 *
 * Scales: a ciphertext's scale is a host double that the caller tracks.
 * Calls that combine ciphertexts (he_add, he_hma_plain, he_hma_scalar,
 * he_conv_convpack) take the scales and return HE_ESCALE when they do not
 * match (two scales match when both are finite and positive and differ by at
 * most 2^-30 relative; both sides compute them with the same IEEE double
 * operations).
 *
 * Errors: each call returns HE_OK (0) or a negative code.  Argument, level,
 * scale and key errors are detected before any launch and leave outputs
 * untouched; he_last_error gives the message.  Launch failures return
 * HE_EDEVICE.
 * Calls enqueue work on the given stream (hipStream_t as void*, NULL = the
 * default stream) and return without synchronising, except where stated.
 * A context is not thread safe: use one per host thread or serialise.
 */
#ifndef FFCONV_HE_H
#define FFCONV_HE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  HE_OK = 0,
  HE_EINVAL = -1,       /* bad argument or shape */
  HE_ELEVEL = -2,       /* level too low/high for the operation */
  HE_ESCALE = -3,       /* scales of the operands do not match */
  HE_ENOKEY = -4,       /* a needed switching key is missing */
  HE_ENOMEM = -5,       /* workspace or device allocation too small / failed */
  HE_EDEVICE = -6,      /* HIP runtime or launch error */
  HE_EUNSUPPORTED = -7  /* parameter combination not built */
};

typedef struct he_ctx he_ctx;

#define HE_MAX_PRIMES 16

typedef struct {
  int32_t n;                      /* ring degree N */
  int32_t n_q;                    /* number of ciphertext primes L (1..15) */
  int32_t q_bits[HE_MAX_PRIMES];  /* bit size of each ciphertext prime (20..61) */
  int32_t p_bits;                 /* bit size of the special prime (20..61) */
} he_params;

/* ---- parameters (host only; no device needed) ----------------------------
 * he_params_moduli: the primes the context would use, written to
 * h_out[0..n_q] (ciphertext primes then P).  A prime of b bits is the
 * largest prime below 2^b that is 1 mod 2N; primes of equal size follow each
 * other downward.  Returns HE_EINVAL for unsupported sizes. */
int he_params_moduli(const he_params *p, uint64_t *h_out);

/* ---- context ---------------------------------------------------------------
 * he_ctx_create builds the prime chain, roots and twiddle tables on the
 * current device (N up to 2^14; larger rings return HE_EUNSUPPORTED).
 * he_ctx_reserve makes sure the workspace holds `bytes` (a library-owned
 * device allocation, replacing a smaller or caller-owned one; call it
 * outside timed regions).  he_ctx_set_workspace hands the context a
 * caller-owned device buffer d_ws of `bytes` (256-byte aligned; NULL and 0
 * detach it) as its workspace; the caller keeps ownership and must keep it
 * alive while the context uses it.  Both wait for the device first and
 * invalidate graphs captured before.  he_ctx_workspace_need returns the bytes
 * the heaviest call on `count` ciphertexts at `level` needs (0 on error). */
int he_ctx_create(const he_params *p, he_ctx **out);
int he_ctx_destroy(he_ctx *ctx);
int he_ctx_reserve(he_ctx *ctx, size_t bytes);
int he_ctx_set_workspace(he_ctx *ctx, void *d_ws, size_t bytes);
size_t he_ctx_workspace_need(const he_ctx *ctx, int count, int level);
int he_ctx_moduli(const he_ctx *ctx, uint64_t *h_out);   /* n_q + 1 values */
const char *he_last_error(const he_ctx *ctx);

/* Schedule knobs of the key switch (the paper does not describe key
 * switching; this library's is hybrid, one digit per ciphertext prime and one
 * special prime P).  The knobs change no result bit, only speed.  knob "p_groups": the
 * number of workgroups (1..min(level, 4)) that share the ModUp + inner
 * product into the special prime P at key-switch level `level` (1..L);
 * value 0 restores the built-in cost model.  knob "split_streams" (level
 * ignored; 1 by default, 0 or 1): run the rotate-and-sum of a DensePack
 * layer's outputs as independent chains on as many streams (each with its
 * own workspace share).  knob "split_parts" (level ignored; 2 by default,
 * 2..4): the number of those chains (fewer when a chunk has under 32 outputs
 * per chain).  knob "modup_halves" at
 * key-switch level `level` (0: every level; -1 restores the default, which is
 * 1 for N >= 8192, else 0): 1 runs ModUp as two half-ring workgroups per
 * target (N >= 2048; a launch follows its largest level), 0 as one workgroup
 * per target.  knob "moddown_halves" (level ignored; -1 restores the default,
 * which is 1 for N >= 16384, else 0): 1 runs a key switch's ModDown as two
 * half-ring workgroups per output limb (N >= 2048; not inside rotate-and-sum
 * chains that keep packed accumulators or write the next step's digits),
 * 0 as one.  knob "hoist_fused" (level ignored; 0 by default, 0 or 1): in
 * he_rotate_hoisted, compute each rotation's inner-product rows inside its
 * ModDown (1) or write them to the workspace first (0).  knob
 * "hoist_pipeline" (level ignored; 0 by default, 0 or 1): hoisted rotations
 * (he_rotate_hoisted(_batch) and the layers built on them) with 64 or more
 * rotations whose temporaries all fit run as up to four chunks, the inner
 * products of one chunk on the call's stream while the previous chunk's
 * P INTT and ModDown run on a second stream.  he_ctx_set_tuning returns
 * HE_EINVAL for an unknown knob or out-of-range level/value;
 * he_ctx_get_tuning returns the value in effect (>= 0) or a negative code. */
int he_ctx_set_tuning(he_ctx *ctx, const char *knob, int level, int value);
int he_ctx_get_tuning(const he_ctx *ctx, const char *knob, int level);

/* ---- ring transforms (the negacyclic NTT that sits inside every Rot and
 * Square) ---------------------------------------------------------------------
 * In place on d_polys = [n_polys][n_limbs][N]; limb t of each poly uses
 * modulus index first_mod + t.  he_ntt maps coefficients to evaluations,
 * he_intt maps back.  Inputs must be reduced (< modulus). */
int he_ntt(he_ctx *ctx, uint64_t *d_polys, int n_polys, int n_limbs, int first_mod, void *stream);
int he_intt(he_ctx *ctx, uint64_t *d_polys, int n_polys, int n_limbs, int first_mod, void *stream);

/* ---- elementwise operations (AddCC and MulPC of Table I) -------------------
 * he_add:  d_out[i] = d_a[i] + d_b[i] for `count` ciphertexts at `level`
 *          (d_out may alias d_a or d_b); HE_ESCALE unless scale_a and
 *          scale_b match.  The sum has that scale.
 * he_hma_plain: one accumulator ciphertext d_acc ([2][level][N]) gets
 *          (accumulate ? d_acc : 0) + sum_{i<k} d_cts[i] * sigma_{g_i}(pt_i),
 *          where d_cts = [k][2][level][N], pt_i starts at
 *          d_pts + i * pt_stride * pt_limbs * N (pt_stride counts whole
 *          plaintexts of pt_limbs limbs; 0 reuses one plaintext), each
 *          plaintext has pt_limbs >= level limbs of which the first `level`
 *          are used, and g_i = h_galois[i] (h_galois NULL: no permutation).
 *          This is MulPC with the plaintext slot rotation folded into its
 *          load.  Scales: every d_cts[i] has ct_scale and every plaintext
 *          pt_scale; with accumulate, *io_acc_scale (the accumulator's scale)
 *          must match ct_scale * pt_scale (else HE_ESCALE); on success
 *          *io_acc_scale = ct_scale * pt_scale.
 * he_hma_scalar: d_acc = (accumulate ? d_acc : 0) + sum_{i<k} w_i * d_cts[i]
 *          with exact signed integers h_w[i] (|w| < 2^62, else HE_EINVAL)
 *          that carry the scale w_scale (e.g. round(x * 2^12) carries 2^12);
 *          scales as for he_hma_plain with pt_scale = w_scale. */
int he_add(he_ctx *ctx, uint64_t *d_out, const uint64_t *d_a, const uint64_t *d_b,
           int count, int level, double scale_a, double scale_b, void *stream);
int he_hma_plain(he_ctx *ctx, uint64_t *d_acc, const uint64_t *d_cts, int k,
                 const uint64_t *d_pts, int pt_stride, int pt_limbs,
                 const int32_t *h_galois, int level, int accumulate,
                 double ct_scale, double pt_scale, double *io_acc_scale, void *stream);
int he_hma_scalar(he_ctx *ctx, uint64_t *d_acc, const uint64_t *d_cts, int k,
                  const int64_t *h_w, int level, int accumulate,
                  double ct_scale, double w_scale, double *io_acc_scale, void *stream);

/* ---- rescale -----------------------------------------------------------------
 * d_out[i] ([2][level-1][N]) = round(d_in[i] / q_{level-1}) for `count`
 * ciphertexts: c_t <- (c_t - centred(c mod q_{level-1})) * q_{level-1}^-1.
 * The caller divides its scale by q_{level-1}.  level >= 2; d_out must not
 * alias d_in. */
int he_rescale(he_ctx *ctx, uint64_t *d_out, const uint64_t *d_in, int count, int level, void *stream);

/* ---- keys ------------------------------------------------------------------
 * In the paper's setting (Section 1, Section 3) the client keeps the secret
 * and the server sees only ciphertexts, plaintext weights and the public
 * switching keys the client sends it.  Key layout (the exchange format):
 * one key = [L][2][L+1][N] canonical uint64 residues, for digit j < L the
 * pair (b_j, a_j) over the moduli q_0 .. q_{L-1}, P, in the NTT domain, with
 *   b_j = -a_j * s + e_j + [t == j] (P mod q_t) s'   (mod modulus t),
 * s' = sigma_g(s) for Galois element g (odd, 1 < g < 2N; rotation left by k
 * uses g = 5^k mod 2N) or s^2 for the relinearisation key (g = 0).
 *
 * he_keys_upload (server side): copies n_keys such keys, keys =
 *          [n_keys][L][2][L+1][N] (host memory, or device memory when
 *          keys_on_device != 0), for Galois elements h_galois[0..n_keys)
 *          into the context's device-resident key store (replacing keys of
 *          the same elements, which invalidates graphs captured before).
 *          Returns HE_EINVAL for a bad or repeated element or a residue not
 *          below its modulus (the store is then unchanged).  Synchronises.
 * he_keys_free: drops the keys of h_galois[0..n_keys) (n_keys == 0: all);
 *          HE_ENOKEY, dropping none, if one is missing.  Waits for the device;
 *          invalidates graphs captured before.
 * he_has_key: 1 if the key of `galois` is stored, else 0.
 * he_keygen_switch (client side, needs the secret; any context with the same
 *          parameters): writes the key of `galois` in the exchange layout to
 *          caller memory d_key ([L][2][L+1][N]) from
 *            d_s  the secret in the NTT domain, [L+1][N] (all moduli),
 *            d_a  uniform residues, NTT domain, [L][L+1][N] (one row per digit),
 *            d_e  signed error coefficients, int64 [L][N].
 *          It stores nothing in the context; synchronises. */
int he_keys_upload(he_ctx *ctx, const int32_t *h_galois, int n_keys, const uint64_t *keys, int keys_on_device,
                   void *stream);
int he_keys_free(he_ctx *ctx, const int32_t *h_galois, int n_keys);
int he_has_key(const he_ctx *ctx, int32_t galois);
int he_keygen_switch(he_ctx *ctx, int32_t galois, const uint64_t *d_s, const uint64_t *d_a, const int64_t *d_e,
                     uint64_t *d_key, void *stream);

/* ---- client helpers (not on the server path) -------------------------------
 * he_from_signed: d_out [n_limbs][N] = d_coeffs (int64 [N]) mod modulus index
 *          first_mod + t, coefficient domain (follow with he_ntt).
 * he_encrypt_sk: d_ct ([2][level][N]) = (-a*s + e + pt, a) with d_pt
 *          [level][N] (NTT), d_a [level][N] (NTT), d_e int64 [N], d_s [L+1][N].
 * he_decrypt: d_out [level][N] (NTT) = c0 + c1*s.
 * he_encode_coeffs: host FP64 encoder; h_out[N] (int64) =
 *          round-half-away(scale * m_k) for the real slot vector h_z
 *          (n_values <= N/2, zero padded); returns HE_EINVAL if any value
 *          reaches 2^62.
 * he_decode_coeffs: host decoder; h_z[n_values] = real slot values of the
 *          real coefficient vector h_m (already divided by the scale). */
int he_from_signed(he_ctx *ctx, uint64_t *d_out, const int64_t *d_coeffs, int n_limbs, int first_mod, void *stream);
int he_encrypt_sk(he_ctx *ctx, uint64_t *d_ct, const uint64_t *d_pt, const uint64_t *d_a,
                  const int64_t *d_e, const uint64_t *d_s, int level, void *stream);
int he_decrypt(he_ctx *ctx, uint64_t *d_out, const uint64_t *d_ct, const uint64_t *d_s, int level, void *stream);
int he_encode_coeffs(int n, const double *h_z, int n_values, double scale, int64_t *h_out);
int he_decode_coeffs(int n, const double *h_m, int n_values, double *h_z);

/* ---- rotations (Rot of Table I) --------------------------------------------
 * he_rotate: d_out[i] = Rot(d_in[i], k) (slot rotation left by k) for
 *          `count` ciphertexts at `level`, all with the key of 5^k mod 2N;
 *          one key switch each: digits of sigma_g(c1) centred per prime,
 *          lifted to every prime and P, inner product with the key, ModDown.
 *          d_out may alias d_in.
 * he_rotate_hoisted: m rotations of ONE ciphertext d_in by h_steps[0..m)
 *          sharing one digit decomposition (the Galois permutation is applied
 *          to the lifted digits); d_outs = [m][2][level][N].  Results are
 *          bit-identical to he_rotate.
 * he_rotate_hoisted_batch: the same for `count` ciphertexts d_in
 *          ([count][2][level][N]) and 1 <= m <= 64 steps: d_outs[i][r] =
 *          Rot(d_in[i], h_steps[r]), [count][m][2][level][N]; one
 *          decomposition per input ciphertext, all of them in a few shared
 *          launches.  Bit-identical to he_rotate.  HE_EINVAL for a step
 *          that is 0 mod N/2, HE_ENOKEY for a missing key (before any
 *          launch); d_outs must not overlap d_in.
 * he_rotsum: in place, for j < r_steps: t <- t + Rot(t, 2^j), for `count`
 *          ciphertexts (the DensePack dot-product sum, Fig. 1b). */
int he_rotate(he_ctx *ctx, uint64_t *d_out, const uint64_t *d_in, int count, int level, int k, void *stream);
int he_rotate_hoisted(he_ctx *ctx, const uint64_t *d_in, int level, const int32_t *h_steps, int m,
                      uint64_t *d_outs, void *stream);
int he_rotate_hoisted_batch(he_ctx *ctx, const uint64_t *d_in, int count, int level, const int32_t *h_steps, int m,
                            uint64_t *d_outs, void *stream);
int he_rotsum(he_ctx *ctx, uint64_t *d_cts, int count, int level, int r_steps, void *stream);

/* ---- allocation-free rotation ----------------------------------------------
 * For callers that cannot allocate device memory at call time (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * he_rotate_static computes exactly what he_rotate computes (same kernels,
 * same bits) but takes its key-switch temporaries (job table, digits, inner
 * products, P-limb coefficients) from a fixed 32 MiB device array of the
 * library, one per GPU, created when the library is loaded on that GPU and
 * held until the process ends.  It never touches the context workspace and
 * calls no allocating routine.  The caller passes inputs and outputs as for
 * he_rotate; the context's device must be current (else HE_EINVAL).  Batches
 * larger than the array run in chunks of he_rotate_static_max_batch(ctx,
 * level) ciphertexts; a level whose single-ciphertext temporaries exceed the
 * array returns HE_ENOMEM before any launch.  Every call on one GPU, from any
 * context or thread, shares that GPU's array: calls whose work overlaps on the
 * device (different streams, or host threads without ordering) race and must
 * be serialised by the caller.  Nothing in the array needs to start at zero;
 * it keeps whatever the last call left there. */
int he_rotate_static(he_ctx *ctx, uint64_t *d_out, const uint64_t *d_in, int count, int level, int k, void *stream);
int he_rotate_static_max_batch(const he_ctx *ctx, int level);

/* ---- batched calls over ragged batches --------------------------------------
 * Each item has its own device pointers and level (host arrays of `count`
 * entries); all items of a call run in one launch per kernel, so work from
 * different layers, requests or levels shares launches.
 * he_batch_rotate: d_outs[b] ([2][level_b][N]) = Rot(d_ins[b], h_steps[b])
 *          (step 0 copies), or d_ins[b] + Rot(d_ins[b], step) when
 *          accumulate != 0; d_outs[b] may alias d_ins[b].
 * he_batch_rescale: d_outs[b] = rescale of d_ins[b] from level_b to
 *          level_b - 1 (level_b >= 2, no aliasing).
 * he_batch_mul_plain: d_outs[b] = d_cts[b] * d_pts[b] slot-wise (MulPC),
 *          d_pts[b] = [level_b][N] NTT-domain plaintext. */
int he_batch_rotate(he_ctx *ctx, uint64_t *const *h_outs, const uint64_t *const *h_ins, const int32_t *h_levels,
                    const int32_t *h_steps, int count, int accumulate, void *stream);
int he_batch_rescale(he_ctx *ctx, uint64_t *const *h_outs, const uint64_t *const *h_ins, const int32_t *h_levels,
                     int count, void *stream);
int he_batch_mul_plain(he_ctx *ctx, uint64_t *const *h_outs, const uint64_t *const *h_cts,
                       const uint64_t *const *h_pts, const int32_t *h_levels, int count, void *stream);

/* ---- CP -> DP combine (Table III, CP-HI2C-DP) ------------------------------
 * O_c channel ciphertexts in ConvPack form (channel o holds its S values in
 * slots 0..S-1, zeros elsewhere), d_in = [o_c][2][level][N], are packed into
 * ceil(O_c / B) DensePack ciphertexts (B = per_dense channels each):
 * dense_m = sum_{o in block m} Rot(Z_o, -(o mod B) * S), so channel o lands
 * at slots (o mod B) * S .. + S - 1 of dense ciphertext o / B.  Needs the
 * rotation keys of -k*S, 0 < k < B; B*S <= N/2.
 * d_out = [ceil(o_c / B)][2][level][N]. */
int he_combine_cp_dp(he_ctx *ctx, const uint64_t *d_in, int o_c, int level, int spatial, int per_dense,
                     uint64_t *d_out, void *stream);
/* The same for `count` independent items in one batched key switch:
 * d_in [count][o_c][2][level][N] -> d_out [count][ceil(o_c/B)][2][level][N]. */
int he_combine_cp_dp_batch(he_ctx *ctx, int count, const uint64_t *d_in, int o_c, int level, int spatial,
                           int per_dense, uint64_t *d_out, void *stream);

/* ---- one-hot gather (the DP->CP step of Table III, and the arrangement of
 * DensePack's replicated outputs into one DensePack ciphertext) ---------------
 * d_out[z] = sum_{k < K} d_cts[z*K + k] * sigma_{5^-k}(E) for z < count,
 * where E = d_mask is a plaintext [level][N] that is one-hot at slot 0:
 * ciphertext k of each group lands at slot k.  d_cts [count*K][2][level][N],
 * d_out [count][2][level][N]; K <= N/2.  No rescale. */
int he_gather_onehot(he_ctx *ctx, int count, const uint64_t *d_cts, int k, const uint64_t *d_mask, int level,
                     uint64_t *d_out, void *stream);

/* ---- square (the x^2 activation, Section 2.1) ------------------------------
 * d_out[i] = relinearised (c0^2, 2 c0 c1) + KeySwitch(c1^2) under the key for
 * s^2, for `count` ciphertexts; the scale squares (no rescale). */
int he_square(he_ctx *ctx, uint64_t *d_out, const uint64_t *d_in, int count, int level, void *stream);

/* ---- convolution layers ----------------------------------------------------
 * Geometry: input X[h][w][c], filters [kh][kw][c][o], output [i][j][o] with
 * out_h = (h + 2 pad - d) / stride + 1 (same for w); S = out_h * out_w.
 * DensePack layout (Section 3.2): X value (h, w, c) sits at slot
 * (c mod B) * H * W + h * W + w of input ciphertext c / B, where
 * B = min(c_in, floor((N/2) / (H*W))) channels fit one ciphertext;
 * M = ceil(c_in / B) input ciphertexts.
 * Border classes: the valid filter-row ranges [lo, hi) are numbered in order
 * of first appearance over output rows 0..out_h-1, likewise columns; class =
 * row_class * n_col_classes + col_class.  Base filter plaintext
 * (o, class, m) carries W[kh][kw][c][o] at slot (c mod B)*H*W + kh*W + kw for
 * the taps valid in that class (zero elsewhere).
 */
typedef struct {
  int32_t h, w, c_in;   /* input tensor */
  int32_t d, stride, pad;
  int32_t o_c;          /* output channels of this DensePack layer */
  int32_t r_steps;      /* rotate-and-sum steps (log2(N/2) sums every slot) */
} he_conv_desc;

/* he_conv_densepack (Table I): for every output value (o, i, j), index
 * o*S + i*out_w + j, computes sum_m x_m * sigma_{g}(F[o][class(i,j)][m]) with
 * g = 5^(-anchor) (rotation right by anchor = (stride i - pad) W +
 * (stride j - pad)), then r_steps rotate-and-add steps, then one rescale.
 *   d_in:   [M][2][level][N]
 *   d_filt: [o_c][n_classes][M][level][N] base filters (NTT domain)
 *   d_out:  [o_c * S][2][level-1][N]: each output replicated in every slot.
 * Needs rotation keys for 2^j, j < r_steps, and workspace for o_c*S
 * ciphertexts at `level` (see he_ctx_workspace_need). */
int he_conv_densepack(he_ctx *ctx, const uint64_t *d_in, int level, const he_conv_desc *desc,
                      const uint64_t *d_filt, uint64_t *d_out, void *stream);
/* The same layer on n_layers independent inputs in one batch (every key
 * switch over all of them): input l at d_in + l * in_stride, its base
 * filters at d_filt + l * filt_stride (0: one filter set shared by all, as
 * when many requests run one model); d_out [n_layers * o_c * S][2][level-1][N]. */
int he_conv_densepack_batch(he_ctx *ctx, int n_layers, const uint64_t *d_in, size_t in_stride, int level,
                            const he_conv_desc *desc, const uint64_t *d_filt, size_t filt_stride, uint64_t *d_out,
                            void *stream);

/* he_conv_convpack (Table II): K channel ciphertexts in, O_c out:
 * d_out[o] = rescale(sum_k round-half-away(h_w[k*o_c + o] * w_scale) * d_in[k])
 * with w_scale = q_{level-1} * target_scale / in_scale (IEEE double, in that
 * order), so the rescale lands on the target: *out_scale = in_scale *
 * w_scale / q_{level-1}.  d_in [K][2][level][N] all at in_scale, d_out
 * [o_c][2][level-1][N].  HE_ELEVEL unless 2 <= level <= L; HE_ESCALE when a
 * scale is not finite and positive or w_scale < 1; HE_EINVAL when a weight
 * times w_scale is not finite or reaches 4e18.  Counts: O_c K MulPC and
 * O_c (K - 1) AddCC. */
int he_conv_convpack(he_ctx *ctx, const uint64_t *d_in, int k, int level, const double *h_w,
                     int o_c, double in_scale, double target_scale, uint64_t *d_out, double *out_scale,
                     void *stream);

/* ---- tap-style DensePack (hoisted rotations) ---------------------------------
 * A variant of the DensePack conv of Table I / Sec. 3.2 that is not in the
 * paper: instead of one rotate-and-sum chain of R rotations per output, each
 * input ciphertext is rotated once per filter tap, all its rotations sharing
 * one digit decomposition (hoisting), and plaintexts holding each tap's
 * weights at the output slots combine them.
 *   desc:   geometry (h, w, c_in, d, stride, pad; o_c outputs; r_steps
 *           unused).  Needs d <= h, d <= w, d^2 <= 64, 2 pad <= d - 1,
 *           h w <= N/2 (else HE_EINVAL).
 *   d_in:   [n_batch][M][2][level][N], the DensePack layout of each input
 *           (B = min(floor(N / (2 h w)), c_in) channels per ciphertext,
 *           channel c = m B + b in block b at slots b h w + y w + x;
 *           M = ceil(c_in / B)), all at in_scale.
 *   d_filt: [o_c][M][d^2][pt_limbs][N] NTT-domain plaintexts (first `level`
 *           limbs used) at pt_scale: plaintext (o, m, t = kh d + kw) holds
 *           W[kh][kw][m B + b][o] in block b at the slot (s i) w + s j of
 *           every output (i, j) whose tap (kh, kw) lies inside the image,
 *           zero elsewhere.
 *   d_filt_p: NULL, or the same plaintexts' residues modulo the special
 *           prime P ([o_c][M][d^2][N], NTT domain): then the ModDown of the
 *           hoisted rotations is deferred past the products (double
 *           hoisting): the key inner products over (Q, P), with
 *           P sigma_t(c0) added, and P x for the zero shift, are multiplied
 *           and summed over (Q, P), and each output takes one ModDown
 *           (exact because ModDown(P a + b) = a + ModDown(b)); with NULL
 *           every rotation takes its own ModDown first.  The two give
 *           different rounding, the same value within noise.
 *   1. x_m rotated left by every nonzero tap shift (kh - pad) w + (kw - pad)
 *      (mod N/2), hoisted per input ciphertext (the zero shift is x_m; see
 *      d_filt_p for where the ModDown goes);
 *   2. t_o = sum_m sum_t d_filt[o][m][t] * Rot(x_m, shift_t);
 *   3. blocks summed into block 0 by the binary method over the bits of B
 *      below the leading one: "double" S <- S + Rot(S, k h w) (k -> 2k),
 *      "inc" S <- t_o + Rot(S, h w) (k -> k + 1); no slot wraps;
 *   4. one rescale.
 * he_conv_tap: d_out [n_batch][o_c][2][level-1][N], output (i, j) of channel
 *          o at slot (s i) w + s j (other slots hold partial sums);
 *          *out_scale = in_scale * pt_scale / q_{level-1}.  Needs rotation
 *          keys for the nonzero tap shifts and for the block steps.  Counts
 *          per input: Rot M (#nonzero shifts) + o_c (#block steps), MulPC
 *          o_c M d^2, AddCC o_c (M d^2 - 1 + #block steps), o_c rescales.
 *          HE_ELEVEL unless 2 <= level <= L; HE_ESCALE for a scale that is
 *          not finite and positive; HE_EINVAL when pt_limbs < level or a
 *          batch needs more than 65535 outputs.
 * ffconv_layer_tap: FFConv with W1 (desc->o_c = r) as he_conv_tap with
 *          plaintexts d_w1 (and d_w1_p, as d_filt_p) at w1_scale, then the
 *          second half of the FFConv
 *          layer with one ciphertext per channel: G_c = y_c * E (d_mask: E,
 *          one at every output slot, NTT domain, >= level-1 limbs, at
 *          mask_scale; it clears the partial sums), Z_o = sum_c
 *          round-half-away(h_w2[c*o_c2 + o] 2^k_bits) G_c (or the same
 *          integers from d_w2_tab, he_int_weight_table's table of the r x o_c2
 *          W2 at level - 1, when d_w2_tab is not NULL: then the call copies
 *          nothing from the host and can be captured in a graph), rescale, and with
 *          `square` x^2 relinearised and rescaled.  d_out: [n_batch][o_c2][2]
 *          [level-2 (-1 more if square)][N], output (i, j) at slot
 *          (s i) w + s j, zero elsewhere; *out_scale = ((in_scale w1_scale /
 *          q_{level-1}) mask_scale 2^k / q_{level-2}) (squared and divided by
 *          q_{level-3} with square).  HE_ELEVEL unless level >= 3 (4 with
 *          square); HE_ENOKEY without the relinearisation key when square.
 * he_tap_workspace_need: workspace bytes for either call (o_c2 = 0: the
 *          conv alone); 0 for a bad geometry or level. */
size_t he_tap_workspace_need(he_ctx *ctx, int n_batch, int level, const he_conv_desc *desc, int o_c2, int square);
int he_conv_tap(he_ctx *ctx, int n_batch, const uint64_t *d_in, int level, const he_conv_desc *desc,
                const uint64_t *d_filt, int pt_limbs, const uint64_t *d_filt_p, double in_scale, double pt_scale,
                uint64_t *d_out, double *out_scale, void *stream);
int ffconv_layer_tap(he_ctx *ctx, int n_batch, const uint64_t *d_in, int level, const he_conv_desc *desc,
                     const uint64_t *d_w1, int w1_limbs, const uint64_t *d_w1_p, double in_scale, double w1_scale,
                     const uint64_t *d_mask, double mask_scale, const double *h_w2, const uint64_t *d_w2_tab,
                     int o_c2, int k_bits, int square, uint64_t *d_out, double *out_scale, void *stream);

/* ---- homomorphic Im2Col for d > 1 (Table III, CP-HI2C-CP / CP-HI2C-DP) -----
 * he_him2col: the K = d^2 I_c ConvPack input ciphertexts of Eq. 1 from a
 *          DensePack input (layout as for he_conv_tap; same geometry limits,
 *          and at most 65 channels per ciphertext).  The paper gives only
 *          the counts; this algorithm:
 *   1. z[m][b] = Rot(x_m, b h w), 0 < b < B_m (B_m channels in x_m), hoisted
 *      per input ciphertext; z[m][0] = x_m;
 *   2. each z[m][b] rotated by every nonzero tap shift (kh - pad) w +
 *      (kw - pad), hoisted per z[m][b];
 *   3. ciphertext k = (kh d + kw) c_in + c (c = m B + b, tap t = kh d + kw)
 *      = mask_t * Rot(z[m][b], shift_t), d_masks [d^2][mask_limbs][N]
 *      (first `level` limbs used, NTT domain, at mask_scale): mask t is one
 *      at the slot (s i) w + s j of every output (i, j) whose tap t lies
 *      inside the image, zero elsewhere;
 *   4. one rescale of each.
 *   d_in [n_batch][M][2][level][N] at in_scale; d_out
 *   [n_batch][K][2][level-1][N], output (i, j)'s pixel under the tap at slot
 *   (s i) w + s j, zero elsewhere; *out_scale = in_scale mask_scale /
 *   q_{level-1}.  Needs rotation keys for the block shifts and the nonzero
 *   tap shifts.  Counts per input: Rot sum_m (B_m - 1 + B_m #nonzero
 *   shifts), MulPC K, K rescales.  HE_ELEVEL unless 2 <= level <= L;
 *   HE_EINVAL for mask_limbs < level or more than 65535 outputs per call.
 * he_him2col_workspace_need: its workspace bytes (0: bad geometry or level). */
size_t he_him2col_workspace_need(he_ctx *ctx, int n_batch, int level, const he_conv_desc *desc);
int he_him2col(he_ctx *ctx, int n_batch, const uint64_t *d_in, int level, const he_conv_desc *desc,
               const uint64_t *d_masks, int mask_limbs, double in_scale, double mask_scale, uint64_t *d_out,
               double *out_scale, void *stream);

/* ffconv_layer_convpack (Section 4.2.2 "ConvPack for W1", Fig. 5; CP-HI2C-CP
 * with d = 1 in Tables III and IX): FFConv with both factors under ConvPack,
 * no rotation at all.
 *   d_in: the K = d^2 I_c Im2Col ciphertexts of the input, [K][2][level][N]
 *         at in_scale (the client packs column k of Eq. 1's matrix I -- the
 *         S = O_w O_h pixels under tap k = (kh d + kw) I_c + c, zero outside
 *         the image -- into slots 0..S-1 of ciphertext k);
 *   h_w1: W1 as the K x r matrix of Eq. 1 (row-major), h_w2: W2 as r x o_c.
 *   1. W1 under ConvPack (he_conv_convpack, landing on target_scale): r
 *      channel ciphertexts at level-1, channel c's S outputs in slots 0..S-1;
 *   2. these are already the per-channel inputs of the 1 x 1 W2 (HGrouping
 *      with d = 1 moves no slot);
 *   3. W2 under ConvPack, landing on target_scale, or with `square` on
 *      sqrt(q_{level-3} target_scale); 4. if square: x^2 (relinearised,
 *      rescaled) back at target_scale.
 * d_out: [o_c][2][level-2 (-1 more if square)][N]; *out_scale its scale.
 * Counts: MulPC r (K + o_c) (integer-scalar products), AddCC r (K - 1) +
 * o_c (r - 1), no Rot.  HE_ELEVEL unless level >= 3 (4 with square);
 * HE_ESCALE / HE_EINVAL as he_conv_convpack for either factor; HE_ENOKEY
 * without the relinearisation key when square. */
int ffconv_layer_convpack(he_ctx *ctx, const uint64_t *d_in, int k, int level, const double *h_w1, int r,
                          const double *h_w2, int o_c, double in_scale, double target_scale, int square,
                          uint64_t *d_out, double *out_scale, void *stream);

/* ffconv_layer (Section 4, DP-HI2C-CP of Table IX):
 *   1. W1 under DensePack exactly as he_conv_densepack (desc->o_c = rank r),
 *      giving r*S replicated ciphertexts at level-1;
 *   2. DP->CP gather: G_c = sum_p y_{c,p} * sigma_{5^-p}(E), E = d_mask (the
 *      one-hot slot-0 plaintext, [level-1][N]), p = i*out_w + j;
 *   3. 1x1 ConvPack: Z_o = sum_c round-half-away(h_w2[c*o_c2 + o] * 2^k_bits) G_c;
 *   4. rescale; 5. if square: Z <- rescale(relinearised Z^2).
 * d_out: [o_c2][2][level-2 (-1 more if square)][N].  The mask is encoded by
 * the caller at scale q_{level-2} * target / (y_scale * 2^k_bits).  A W2
 * weight times 2^k_bits that is not finite or reaches 4e18 returns HE_EINVAL
 * before any launch. */
int ffconv_layer(he_ctx *ctx, const uint64_t *d_in, int level, const he_conv_desc *desc,
                 const uint64_t *d_w1_filt, const uint64_t *d_mask, const double *h_w2, int o_c2,
                 int k_bits, int square, uint64_t *d_out, void *stream);

/* he_int_weight_table: the exact integer weights round-half-away(h_w[i] *
 * 2^k_bits), i < count, as residues for limbs < level followed by their
 * Shoup companions, written to caller-owned device memory d_tab
 * (2 * count * level uint64, laid out [2][count][level]).  The 1x1 ConvPack
 * weights of ffconv_layer_batch (W2 of one layer, count = r * o_c2, row-major
 * [r][o_c2], at level - 1) use this form.  Copies through pinned host memory
 * on `stream`; not capturable in a graph. */
int he_int_weight_table(he_ctx *ctx, const double *h_w, int count, int k_bits, int level, uint64_t *d_tab,
                        void *stream);

/* ffconv_layer_batch: n_layers independent FFConv layers of one geometry
 * (batched serving, and Sec. 4's layer run many times), as ffconv_layer on
 * each, with every key switch batched over all layers' ciphertexts (one
 * Galois key read per rotate-and-add step for all of them).  Layer l reads
 * its input ciphertext at d_in + l * in_stride, its W1 base filters at
 * d_w1_filt + l * filt_stride and its W2 table (he_int_weight_table) at
 * d_w2_tab + l * 2 * r * o_c2 * (level - 1) (strides in uint64); the mask is
 * shared.  d_out: [n_layers][o_c2][2][..][N].  n_layers * max(r, o_c2) <=
 * 65535.  Makes no host-to-device copies, so it can be captured in a graph.
 * Workspace: he_ffconv_workspace_need. */
int ffconv_layer_batch(he_ctx *ctx, int n_layers, const uint64_t *d_in, size_t in_stride, int level,
                       const he_conv_desc *desc, const uint64_t *d_w1_filt, size_t filt_stride,
                       const uint64_t *d_mask, const uint64_t *d_w2_tab, int o_c2, int square, uint64_t *d_out,
                       void *stream);

/* ---- pieces of a layer for iteration-level (continuous) batching -----------
 * A serving engine that merges the work of requests at different points of
 * their nets into shared launches runs a DensePack layer as its three parts:
 * he_densepack_hma: the MulPC of he_conv_densepack_batch only (Table I's
 *          O MulPC): d_acc [n_layers * o_c * S][2][level][N] gets the
 *          unsummed products at `level` (no rotation, no rescale).
 * he_rotsum_groups: one rotate-and-add step for several groups of such
 *          accumulators at once: for every group g and i < count_g,
 *          acc_g[i] <- acc_g[i] + Rot(acc_g[i], 2^step_g) in place (each
 *          group its own level and step, so chains that started at
 *          different times share the launch; R steps j = 0..R-1 complete
 *          the DensePack sum of Fig. 1b).  Needs the keys of 2^step_g;
 *          2^step a multiple of N/2 is refused (identity).
 * ffconv_tail_batch: the rest of ffconv_layer_batch after the rotate-and-
 *          sum: rescale of the n_layers * r * S summed accumulators d_acc
 *          (r = desc->o_c, at `level`), DP->CP gather with d_mask, 1x1
 *          ConvPack with the W2 tables d_w2_tab (he_int_weight_table, layer l
 *          at d_w2_tab + l * 2 * r * o_c2 * (level - 1)), rescale, and with
 *          `square` x^2 + relinearisation + rescale.  d_out as
 *          ffconv_layer_batch's.
 * Results are bit-identical to the one-call layers (each ciphertext's
 * arithmetic is independent of what else shares a launch). */
typedef struct {
  uint64_t *acc;   /* [count][2][level][N], device */
  int32_t count;
  int32_t level;
  int32_t step;    /* this group's rotation is by 2^step */
} he_rotsum_group;
int he_densepack_hma(he_ctx *ctx, int n_layers, const uint64_t *d_in, size_t in_stride, int level,
                     const he_conv_desc *desc, const uint64_t *d_filt, size_t filt_stride, uint64_t *d_acc,
                     void *stream);
int he_rotsum_groups(he_ctx *ctx, const he_rotsum_group *h_groups, int n_groups, void *stream);
int ffconv_tail_batch(he_ctx *ctx, int n_layers, const uint64_t *d_acc, int level, const he_conv_desc *desc,
                      const uint64_t *d_mask, const uint64_t *d_w2_tab, int o_c2, int square, uint64_t *d_out,
                      void *stream);

/* Workspace bytes ffconv_layer / ffconv_layer_batch need for n_layers layers
 * (0 on bad arguments); the batch runs in a smaller workspace too, in more
 * chunks, down to one ciphertext's temporaries. */
size_t he_ffconv_workspace_need(const he_ctx *ctx, int n_layers, int level, const he_conv_desc *desc, int o_c2,
                                int square);

/* ---- graphs (HIP graphs instead of per-call launches) ---------------------
 * he_graph_begin starts capturing `stream` (a non-default stream; thread-local
 * capture mode); the library calls made on it until he_graph_end are
 * recorded, not run, and he_graph_end instantiates them.  he_graph_launch
 * replays the whole recorded sequence on `stream` in one launch, with the
 * same device pointers (inputs, outputs, workspace, keys): write new inputs
 * into the same buffers between replays.  It returns HE_EINVAL if the
 * workspace was reallocated or keys were replaced or freed since the capture.
 * Calls that copy host tables (he_int_weight_table, ffconv_layer with host
 * W2, he_batch_*), workspace changes, key upload and key freeing fail with
 * HE_EUNSUPPORTED while capturing.  Replays of one graph must not overlap
 * with each other or with other calls on the context (they share its
 * workspace). */
typedef struct he_graph he_graph;
int he_graph_begin(he_ctx *ctx, void *stream);
int he_graph_end(he_ctx *ctx, void *stream, he_graph **out);
int he_graph_launch(he_graph *graph, void *stream);
int he_graph_destroy(he_graph *graph);

/* Executed operation counters of the last layer call (he_conv_densepack,
 * he_conv_convpack, ffconv_layer): MulPC, AddCC, Rot, rescaled ciphertexts,
 * squares, integer-scalar products. */
typedef struct {
  int64_t mulpc, addcc, rot, rescale, square, scalar_mul;
} he_counts;
int he_last_counts(const he_ctx *ctx, he_counts *out);

/* ---- instrumentation (not part of the evaluated path) ---------------------
 * he_prof_select: from now on every launch of the kernel named `kernel`
 * ("ntt", "ks_digits", "ks_modup_stage" (the ModUp + inner-product work of
 * a key switch: one kernel when the ring's primes span one or two width
 * classes, else one per class on two streams, fork to join),
 * "ks_modup_ip" / "ks_modup_ip_f64" / "ks_modup_ip_wide" (the per-class
 * kernels of the three-class case), "intt_last", "drop_last",
 * "dp_hma", "hma_perm", "scalar_mac", "tensor_sq", "modup_store", "ip_perm",
 * "add") is bracketed by two HIP events recorded on the stream it is launched
 * on (timing-only events without the system-scope fence, so they add no
 * cache write-back between the kernels they bracket); NULL or "" stops
 * recording.  he_prof_read waits for the recorded events and
 * returns the summed kernel time (ms) and the number of launches since the
 * last select or read, then clears them. */
int he_prof_select(he_ctx *ctx, const char *kernel);
int he_prof_read(he_ctx *ctx, double *total_ms, int64_t *launches);
/* he_prof_read_busy: as he_prof_read, plus the time (ms) during which at least
 * one bracketed launch was running (the union of their intervals; launches on
 * two streams overlap, so busy_ms <= total_ms). */
int he_prof_read_busy(he_ctx *ctx, double *total_ms, double *busy_ms, int64_t *launches);

#ifdef __cplusplus
}
#endif
#endif /* FFCONV_HE_H */

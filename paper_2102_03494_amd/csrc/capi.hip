// C-ABI of the homomorphic convolution library: context, keys, workspace,
// argument checks and kernel orchestration.  See include/ffconv_he.h for the
// contract of every entry point.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/ffconv_he.h"
#include "host_params.h"
#include "ctx.h"
#include "kernels_elem.h"

using namespace he;

// Device scratch of the allocation-free rotation (he_rotate_static): one
// array per GPU, created when the library's code object is loaded on that
// GPU and held until the process ends.  Host code never passes the name
// `scratch` to a kernel (on the host it is only a stand-in for the symbol):
// its device address on each GPU comes from hipGetSymbolAddress at context
// creation, with that GPU current, and is kept per device below.
constexpr size_t STATIC_SCRATCH_BYTES = (size_t)32 << 20;
static __device__ __align__(256) unsigned char scratch[STATIC_SCRATCH_BYTES];

namespace {

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
char* g_scratch_addr[MAX_DEVICES] = {};

// Looks up the address of this device's scratch array once per device (the
// device must be current) and stores it in the context.
int scratch_setup(he_ctx* c) {
  if (c->device < 0 || c->device >= MAX_DEVICES) return fail(c, HE_EDEVICE, "device index %d too large", c->device);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_addr[c->device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(c, HE_EDEVICE, "hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
    g_scratch_addr[c->device] = (char*)p;
  }
  c->fixed_scratch = g_scratch_addr[c->device];
  return HE_OK;
}

// Copies `bytes` from host to device memory `dst` on stream s through a ring
// of pinned buffers; a slot is reused only after its previous copy finished.
int upload(he_ctx* c, void* dst, const void* src, size_t bytes, hipStream_t s) {
  if (c->capturing)
    return fail(c, HE_EUNSUPPORTED, "this call copies host tables and cannot be captured in a graph "
                                    "(use the device-table form, e.g. ffconv_layer_batch)");
  StageSlot& st = c->stage[c->stage_next];
  c->stage_next = (c->stage_next + 1) % STAGE_SLOTS;
  if (st.pending) {
    if (hipEventSynchronize(st.ev) != hipSuccess) return fail(c, HE_EDEVICE, "staging event wait failed");
    st.pending = false;
  }
  if (st.cap < bytes) {
    if (st.host) (void)hipHostFree(st.host);
    size_t cap = std::max<size_t>(bytes, 1 << 16);
    if (hipHostMalloc((void**)&st.host, cap, hipHostMallocDefault) != hipSuccess) {
      st.host = nullptr;
      st.cap = 0;
      return fail(c, HE_ENOMEM, "pinned staging allocation failed");
    }
    st.cap = cap;
  }
  if (!st.ev && hipEventCreateWithFlags(&st.ev, hipEventDisableTiming) != hipSuccess)
    return fail(c, HE_EDEVICE, "event create failed");
  std::memcpy(st.host, src, bytes);
  if (hipMemcpyAsync(dst, st.host, bytes, hipMemcpyHostToDevice, s) != hipSuccess)
    return fail(c, HE_EDEVICE, "staging copy failed");
  (void)hipEventRecord(st.ev, s);
  st.pending = true;
  return HE_OK;
}

// ---- shared orchestration ----------------------------------------------------

constexpr int PG_MAX = 4;

// Number of groups the P target's digits are split into at key-switch level
// `level`: set per level through he_ctx_set_tuning, else from a cost model
// that makes a P workgroup about as long as a ciphertext-prime workgroup
// (relative transform cost per class: narrow 1, f64 1.3, wide 3).
int p_groups(const he_ctx* c, int level) {
  if (level < 2) return 1;
  const int lim = std::min(level, PG_MAX);
  if (c->pg_set[level] > 0) return std::min(c->pg_set[level], lim);
  static const double cost[3] = {1.0, 1.3, 3.0};
  double cq = 0;
  for (int t = 0; t < level; ++t) cq += cost[c->mods.m[t].cls];
  cq /= level;
  const double p_block = level * cost[c->mods.m[c->big_l].cls];
  const int pg = (int)std::lround(p_block / ((level - 1) * cq));
  return std::max(1, std::min(pg, lim));
}

// Key-switch scratch per job: digits (lmax), u (2 (lmax + pg)), rc (2).
size_t ks_elems_per_job(int lmax, int pg, int n) { return (3 * (size_t)lmax + 2 * (size_t)pg + 2) * n; }

struct KsScratch {
  KsJob* jobs = nullptr;
  u64 *dcoef = nullptr, *u = nullptr, *rc = nullptr;
  int pg = 1;
};

bool take_scratch(Arena& ar, int count, int lmax, int pg, int n, KsScratch& ks) {
  ks.pg = pg;
  ks.jobs = ar.take<KsJob>(count);
  ks.dcoef = ar.take<u64>((size_t)count * lmax * n);
  ks.u = ar.take<u64>((size_t)count * 2 * (lmax + pg) * n);
  ks.rc = ar.take<u64>((size_t)count * 2 * n);
  return ks.jobs && ks.dcoef && ks.u && ks.rc;
}

// Jobs that fit the arena with key-switch scratch at lmax (+ extra per job).
int chunk_for(Arena& ar, int count, int lmax, int pg, int n, size_t extra_per_job_elems = 0) {
  const size_t per = ks_elems_per_job(lmax, pg, n) + extra_per_job_elems + 128;
  return (int)std::min<size_t>({(size_t)count, ar.left() / 8 / per, (size_t)32000});
}

void make_jobs(he_ctx* c, KsJob* jobs, int count, const u64* d_base, size_t d_stride, const u64* c_base,
               size_t c_stride, u64* out_base, size_t out_stride, const u64* key, u32 g, u32 ginv, int level,
               hipStream_t s, int flags = 0) {
  (void)c;
  k_make_jobs<<<(count + 255) / 256, 256, 0, s>>>(jobs, count, d_base, d_stride, c_base, c_stride, out_base,
                                                  out_stride, key, g, ginv, level, flags);
}

// Rotation (EPI_ROT into out) or rotate-and-add (EPI_ROTSUM, may be in place)
// of `count` ciphertexts at one level by k, chunked to the workspace.
int rotate_batch(he_ctx* c, u64* out, const u64* in, int count, int level, int k, int epi, Arena& ar,
                 hipStream_t s) {
  const int n = c->n;
  const u32 g = galois_of(k, n);
  const u64* key = nullptr;
  if (g != 1) {
    auto it = c->keys.find((int)g);
    if (it == c->keys.end()) return fail(c, HE_ENOKEY, "no rotation key for step %d (Galois element %u)", k, g);
    key = it->second;
  }
  const u32 ginv = galois_of(-k, n);
  const int pg = p_groups(c, level);
  const int chunk = chunk_for(ar, count, level, pg, n);
  if (chunk < 1) return fail(c, HE_ENOMEM, "workspace too small for one key switch at level %d", level);
  Arena sub = ar;
  KsScratch ks;
  if (!take_scratch(sub, chunk, level, pg, n, ks)) return fail(c, HE_ENOMEM, "workspace too small");
  const size_t cstride = (size_t)2 * level * n;
  for (int b0 = 0; b0 < count; b0 += chunk) {
    const int cn = std::min(chunk, count - b0);
    const u64* cin = in + (size_t)b0 * cstride;
    u64* cout = out + (size_t)b0 * cstride;
    make_jobs(c, ks.jobs, cn, cin + (size_t)level * n, cstride, cin, cstride, cout, cstride, key, g, ginv, level, s);
    if (key) dispatch_logn<LKsCore>(c->logn, c, (const KsJob*)ks.jobs, cn, level, pg, ks.dcoef, ks.u, ks.rc, s);
    dispatch_logn<LDrop>(c->logn, c, (int)MODE_P, epi, (const KsJob*)ks.jobs, cn, level, level + pg,
                         (const u64*)ks.u, (const u64*)ks.rc, s);
  }
  return check_launch(c, "rotate");
}

// Rotate-and-sum chain acc <- acc + rot(acc, 2^j), j = 0 .. steps - 1, in
// place over `count` ciphertexts at one level, with the job tables of all
// steps built by one launch (chain_prepare) instead of one per step.
struct Chain {
  KsJob* jobs = nullptr;  // [steps][count]
  KsScratch ks;
  int count = 0, level = 0, pg = 1, steps = 0;
  bool packed = false;  // the accumulator leaves the chain packed
  bool in_packed0 = false;  // the first step reads packed input too
};

// False (nothing launched) when the chain does not fit the arena in one
// chunk or has too many steps; the caller then rotates step by step.
// With in_packed0 (honoured only where the accumulator is kept packed), the
// chain starts from a packed accumulator; ch.in_packed0 says whether it does.
bool chain_prepare(he_ctx* c, u64* acc, int count, int level, int steps, Arena ar, hipStream_t s, Chain& ch,
                   bool in_packed0 = false) {
  const int n = c->n;
  if (steps < 1 || steps > MAX_CHAIN || count < 1) return false;
  const int pg = p_groups(c, level);
  if (chunk_for(ar, count, level, pg, n, (size_t)steps * sizeof(KsJob) / 8 + 1) < count) return false;
  ch.jobs = ar.take<KsJob>((size_t)steps * count);
  if (!ch.jobs || !take_scratch(ar, count, level, pg, n, ch.ks)) return false;
  ChainKeys ck{};
  for (int j = 0; j < steps; ++j) {
    const u32 g = galois_of(1 << j, n);
    auto it = c->keys.find((int)g);
    if (g != 1 && it == c->keys.end()) return false;
    ck.key[j] = (g == 1) ? nullptr : it->second;
    ck.g[j] = g;
    ck.ginv[j] = galois_of(-(1 << j), n);
  }
  ch.count = count;
  ch.level = level;
  ch.pg = pg;
  ch.steps = steps;
  // between steps the accumulator is kept packed when every ciphertext prime is narrow
  ch.packed = c->q_mask == (1u << CLS_N32);
  ch.in_packed0 = ch.packed && in_packed0;
  k_make_chain_jobs<<<dim3((count + 255) / 256, steps), 256, 0, s>>>(ch.jobs, count, acc, (size_t)2 * level * n,
                                                                    (size_t)level * n, level, ck, (int)ch.packed,
                                                                    (int)ch.in_packed0);
  return true;
}

// Step j of the chain.  When steps j and j + 1 both switch keys (and the
// ring is at most 2^NEXT_DIGITS_MAX_LOGN), step j's ModDown also writes step
// j + 1's digits, and step j + 1 launches no digit kernel.
void chain_step(he_ctx* c, const Chain& ch, int j, hipStream_t s) {
  const KsJob* jobs = ch.jobs + (size_t)j * ch.count;
  auto switches = [&](int k) { return k < ch.steps && galois_of(1 << k, c->n) != 1; };
  // ModDown writes the next step's digits only where the kernel has them
  auto fused = [&](int k) { return c->logn <= NEXT_DIGITS_MAX_LOGN && switches(k) && switches(k + 1); };
  // as k_make_chain_jobs sets
  const int pk = ch.packed ? (JOB_OUT_PACKED | ((j > 0 || ch.in_packed0) ? JOB_IN_PACKED : 0)) : 0;
  if (switches(j))
    dispatch_logn<LKsCore>(c->logn, c, jobs, ch.count, ch.level, ch.pg, ch.ks.dcoef, ch.ks.u, ch.ks.rc, s, pk,
                           j > 0 && fused(j - 1));
  NextDigits nd{nullptr, 1u, ch.level};
  if (fused(j)) {
    nd.dcoef = ch.ks.dcoef;
    nd.ginv = galois_of(-(1 << (j + 1)), c->n);
  }
  dispatch_logn<LDrop>(c->logn, c, (int)MODE_P, (int)EPI_ROTSUM, jobs, ch.count, ch.level, ch.level + ch.pg,
                       (const u64*)ch.ks.u, (const u64*)ch.ks.rc, s, pk, nd);
}

// in_packed: the input is packed (narrow limbs as 32-bit words, see KsJob).
int rescale_batch(he_ctx* c, u64* out, const u64* in, int count, int level, Arena& ar, hipStream_t s,
                  bool in_packed = false) {
  const int n = c->n;
  const int chunk = (int)std::min<size_t>({(size_t)count, ar.left() / 8 / (2 * (size_t)n + 64), (size_t)32000});
  if (chunk < 1) return fail(c, HE_ENOMEM, "workspace too small for rescale");
  Arena sub = ar;
  KsJob* jobs = sub.take<KsJob>(chunk);
  u64* rc = sub.take<u64>((size_t)chunk * 2 * n);
  if (!jobs || !rc) return fail(c, HE_ENOMEM, "workspace too small for rescale");
  for (int b0 = 0; b0 < count; b0 += chunk) {
    const int cn = std::min(chunk, count - b0);
    const u64* cin = in + (size_t)b0 * 2 * level * n;
    u64* cout = out + (size_t)b0 * 2 * (level - 1) * n;
    make_jobs(c, jobs, cn, cin, (size_t)2 * level * n, cin, (size_t)2 * level * n, cout,
              (size_t)2 * (level - 1) * n, nullptr, 1u, 1u, level, s, in_packed ? JOB_IN_PACKED : 0);
    const int pk = in_packed ? JOB_IN_PACKED : 0;
    dispatch_logn<LIntt1>(c->logn, c, (const KsJob*)jobs, cn, level, rc, s, pk);
    dispatch_logn<LDrop>(c->logn, c, (int)MODE_LAST, (int)EPI_STORE, (const KsJob*)jobs, cn, level, 0,
                         (const u64*)nullptr, (const u64*)rc, s, pk);
  }
  return check_launch(c, "rescale");
}

int square_batch(he_ctx* c, u64* out, const u64* in, int count, int level, Arena& ar, hipStream_t s) {
  const int n = c->n;
  auto it = c->keys.find(0);
  if (it == c->keys.end()) return fail(c, HE_ENOKEY, "no relinearisation key");
  const int pg = p_groups(c, level);
  const int chunk = chunk_for(ar, count, level, pg, n, 3 * (size_t)level * n);
  if (chunk < 1) return fail(c, HE_ENOMEM, "workspace too small for square");
  Arena sub = ar;
  u64* d01 = sub.take<u64>((size_t)chunk * 2 * level * n);
  u64* d2 = sub.take<u64>((size_t)chunk * level * n);
  KsScratch ks;
  if (!d01 || !d2 || !take_scratch(sub, chunk, level, pg, n, ks)) return fail(c, HE_ENOMEM, "workspace too small");
  for (int b0 = 0; b0 < count; b0 += chunk) {
    const int cn = std::min(chunk, count - b0);
    const u64* cin = in + (size_t)b0 * 2 * level * n;
    u64* cout = out + (size_t)b0 * 2 * level * n;
    {
      Prof pr(c, "tensor_sq", s);
      k_tensor_sq<<<dim3(n / 256, level, cn), 256, 0, s>>>(d01, d2, cin, level, n, c->mods);
    }
    make_jobs(c, ks.jobs, cn, d2, (size_t)level * n, d01, (size_t)2 * level * n, cout, (size_t)2 * level * n,
              it->second, 1u, 1u, level, s);
    dispatch_logn<LKsCore>(c->logn, c, (const KsJob*)ks.jobs, cn, level, pg, ks.dcoef, ks.u, ks.rc, s);
    dispatch_logn<LDrop>(c->logn, c, (int)MODE_P, (int)EPI_RELIN, (const KsJob*)ks.jobs, cn, level, level + pg,
                         (const u64*)ks.u, (const u64*)ks.rc, s);
  }
  return check_launch(c, "square");
}

bool build_geom(he_ctx* c, const he_conv_desc* d, DPGeom& g, int& n_cls) {
  if (!d || d->h < 1 || d->w < 1 || d->c_in < 1 || d->d < 1 || d->stride < 1 || d->pad < 0 || d->o_c < 1 ||
      d->r_steps < 0 || d->r_steps > 20)
    return false;
  g = DPGeom{};
  g.h = d->h; g.w = d->w; g.c_in = d->c_in; g.d = d->d; g.stride = d->stride; g.pad = d->pad; g.o_c = d->o_c;
  g.out_h = (d->h + 2 * d->pad - d->d) / d->stride + 1;
  g.out_w = (d->w + 2 * d->pad - d->d) / d->stride + 1;
  if (g.out_h < 1 || g.out_w < 1 || g.out_h > 64 || g.out_w > 64) return false;
  const int slots = c->n / 2;
  const int plane = d->h * d->w;
  if (plane > slots) return false;
  const int per = std::min(d->c_in, slots / plane);
  g.m_cts = (d->c_in + per - 1) / per;
  auto ranges = [&](int out, int size, int* cls, int& n_cls_axis) {
    std::vector<std::pair<int, int>> seen;
    for (int i = 0; i < out; ++i) {
      int start = d->stride * i - d->pad;
      std::pair<int, int> r(std::max(0, -start), std::min(d->d, size - start));
      auto f = std::find(seen.begin(), seen.end(), r);
      if (f == seen.end()) {
        seen.push_back(r);
        cls[i] = (int)seen.size() - 1;
      } else {
        cls[i] = (int)(f - seen.begin());
      }
    }
    n_cls_axis = (int)seen.size();
  };
  ranges(g.out_h, d->h, g.row_cls, g.n_row_cls);
  ranges(g.out_w, d->w, g.col_cls, g.n_col_cls);
  n_cls = g.n_row_cls * g.n_col_cls;
  g.per_layer = g.out_h * g.out_w * g.o_c;
  g.x_stride = g.f_stride = 0;
  return true;
}

// DensePack conv (HMA + rotate-and-sum + rescale) into d_out, chunked over
// outputs so that any workspace holding one output's temporaries works.
// n_layers independent layers of one geometry: layer l reads its input at
// d_in + l x_stride and its filters at d_filt + l f_stride; the outputs of
// all layers are one batch (layer-major) for every key switch.
int densepack_run(he_ctx* c, const u64* d_in, int level, const he_conv_desc* desc, const u64* d_filt, u64* d_out,
                  Arena& ar, hipStream_t s, int n_layers = 1, size_t x_stride = 0, size_t f_stride = 0) {
  DPGeom geo;
  int n_cls = 0;
  if (!build_geom(c, desc, geo, n_cls)) return fail(c, HE_EINVAL, "bad convolution geometry");
  if (level < 2 || level > c->big_l) return fail(c, HE_ELEVEL, "DensePack needs 2 <= level <= L (got %d)", level);
  const int n = c->n;
  const int spatial = geo.out_h * geo.out_w;
  if ((long long)n_layers * geo.per_layer > (1ll << 30)) return fail(c, HE_EINVAL, "too many outputs");
  geo.x_stride = x_stride;
  geo.f_stride = f_stride;
  const int total = spatial * geo.o_c * n_layers;
  for (int j = 0; j < desc->r_steps; ++j) {
    u32 g = galois_of(1 << j, n);
    if (g != 1 && !c->keys.count((int)g)) return fail(c, HE_ENOKEY, "missing rotation key for step %d", 1 << j);
  }
  // per output: accumulator (2 level N) + key switch temporaries
  const int chunk =
      std::min(chunk_for(ar, total, level, p_groups(c, level), n, (size_t)2 * level * n + 2 * (size_t)n), 16000);
  if (chunk < 1) return fail(c, HE_ENOMEM, "workspace too small for DensePack");
  for (int o0 = 0; o0 < total; o0 += chunk) {
    const int cn = std::min(chunk, total - o0);
    Arena sub = ar;
    u64* acc = sub.take<u64>((size_t)cn * 2 * level * n);
    if (!acc) return fail(c, HE_ENOMEM, "workspace too small");
    u64* out = d_out + (size_t)o0 * 2 * (level - 1) * n;
    const int n_cls = (int)c->has_cls[0] + (int)c->has_cls[1] + (int)c->has_cls[2];
    // The chains' job tables come first, so that the HMA can leave the
    // products packed where the chains keep their accumulators packed.
    const int parts = (c->split_streams && cn >= 64 && n_cls <= 2) ? std::min(c->split_parts, cn / 32) : 1;
    if (parts > 1) {
      // The outputs are independent chains through the rotate-and-add steps:
      // `parts` chains on as many streams fill each other's kernel tails; one
      // fork and one join per chunk, each chain with its own scratch.
      hipStream_t st[MAX_SPLIT] = {s, c->side, c->side_x[0], c->side_x[1]};
      hipEvent_t jn[MAX_SPLIT] = {nullptr, c->join_ev, c->join_x[0], c->join_x[1]};
      int cnt[MAX_SPLIT], first[MAX_SPLIT];
      for (int p = 0; p < parts; ++p) {
        first[p] = (int)((long long)cn * p / parts);
        cnt[p] = (int)((long long)cn * (p + 1) / parts) - first[p];
      }
      Arena ap[MAX_SPLIT] = {sub, sub, sub, sub};
      sub.split(parts, ap);
      Chain ch[MAX_SPLIT];
      bool chained = true;
      for (int p = 0; p < parts && chained; ++p)
        chained = chain_prepare(c, acc + (size_t)first[p] * 2 * level * n, cnt[p], level, desc->r_steps, ap[p], s,
                                ch[p], true);
      dispatch_logn<LDpHma>(c->logn, c, d_in, d_filt, acc, level, o0, cn, geo, s, chained && ch[0].in_packed0);
      (void)hipEventRecord(c->fork_ev, s);
      for (int p = 1; p < parts; ++p) (void)hipStreamWaitEvent(st[p], c->fork_ev, 0);
      int e = HE_OK;
      if (chained) {
        for (int j = 0; j < desc->r_steps; ++j)
          for (int p = 0; p < parts; ++p) chain_step(c, ch[p], j, st[p]);
      } else {
        for (int j = 0; j < desc->r_steps && !e; ++j)
          for (int p = 0; p < parts && !e; ++p) {
            u64* a = acc + (size_t)first[p] * 2 * level * n;
            e = rotate_batch(c, a, a, cnt[p], level, 1 << j, EPI_ROTSUM, ap[p], st[p]);
          }
      }
      for (int p = 0; p < parts && !e; ++p)
        e = rescale_batch(c, out + (size_t)first[p] * 2 * (level - 1) * n, acc + (size_t)first[p] * 2 * level * n,
                          cnt[p], level, ap[p], st[p], chained && ch[p].packed);
      for (int p = 1; p < parts; ++p) {
        (void)hipEventRecord(jn[p], st[p]);
        (void)hipStreamWaitEvent(s, jn[p], 0);
      }
      if (e) return e;
    } else {
      Chain ch;
      const bool chained = chain_prepare(c, acc, cn, level, desc->r_steps, sub, s, ch, true);
      dispatch_logn<LDpHma>(c->logn, c, d_in, d_filt, acc, level, o0, cn, geo, s, chained && ch.in_packed0);
      bool packed = false;
      if (chained) {
        for (int j = 0; j < desc->r_steps; ++j) chain_step(c, ch, j, s);
        packed = ch.packed;
      } else {
        for (int j = 0; j < desc->r_steps; ++j) {
          int e = rotate_batch(c, acc, acc, cn, level, 1 << j, EPI_ROTSUM, sub, s);
          if (e) return e;
        }
      }
      int e = rescale_batch(c, out, acc, cn, level, sub, s, packed);
      if (e) return e;
    }
  }
  c->counts.mulpc += (int64_t)total * geo.m_cts;
  c->counts.addcc += (int64_t)total * (geo.m_cts - 1) + (int64_t)total * desc->r_steps;
  c->counts.rot += (int64_t)total * desc->r_steps;
  c->counts.rescale += total;
  return check_launch(c, "densepack");
}

bool level_ok(he_ctx* c, int level) { return level >= 1 && level <= c->big_l; }

// Scales are host doubles that caller and library compute with the same IEEE
// operations; two scales agree when both are finite and positive and differ
// by at most 2^-30 relative.
bool scale_ok(double a) { return std::isfinite(a) && a > 0; }
bool scales_agree(double a, double b) {
  return scale_ok(a) && scale_ok(b) && std::fabs(a - b) <= std::ldexp(std::max(a, b), -30);
}

// Residue table of signed integer scalars w (count values) for limbs < level,
// laid out [count][level] followed by the Shoup companions.
std::vector<u64> scalar_table(he_ctx* c, const std::vector<int64_t>& w, int level) {
  std::vector<u64> tab(2 * w.size() * level);
  for (size_t k = 0; k < w.size(); ++k) {
    for (int t = 0; t < level; ++t) {
      const u64 r = from_signed(w[k], c->mods.m[t]);
      tab[k * level + t] = r;
      tab[w.size() * level + k * level + t] = shoup_companion(r, c->moduli[t]);
    }
  }
  return tab;
}

int64_t round_half_away(double x) {
  double r = std::floor(std::fabs(x) + 0.5);
  return (int64_t)(x < 0 ? -r : r);
}

// out[l][o] = sum_k w_l[k][o] * in[l][k] for integer weights (no rescale),
// n_layers independent layers: layer l reads K ciphertexts at in + l in_stride
// and its device table (scalar_table layout, 2 K o_c level u64) at
// d_tab + l 2 K o_c level.
int scalar_mac_dev(he_ctx* c, u64* out, const u64* in, int k, const u64* d_tab, int o_c, int level, int n_layers,
                   size_t in_stride, hipStream_t s, bool shared_tab = false) {
  if ((long long)n_layers * o_c > 65535) return fail(c, HE_EINVAL, "too many output ciphertexts for one launch");
  const size_t tab = (size_t)k * o_c * level;
  Prof pr(c, "scalar_mac", s);
  k_scalar_mac<<<dim3(c->n / 256, level, n_layers * o_c), 256, 0, s>>>(out, in, k, o_c, d_tab, d_tab + tab, level,
                                                                       c->n, in_stride, shared_tab ? 0 : 2 * tab,
                                                                       c->mods);
  return check_launch(c, "scalar_mac");
}

// out[o] = sum_k w[k][o] * in[k] for host integer weights (no rescale).
int scalar_mac(he_ctx* c, u64* out, const u64* in, int k, const std::vector<int64_t>& w, int o_c, int level,
               Arena& ar, hipStream_t s) {
  std::vector<u64> tab = scalar_table(c, w, level);
  u64* d_tab = ar.take<u64>(tab.size());
  if (!d_tab) return fail(c, HE_ENOMEM, "workspace too small for weight table");
  int e = upload(c, d_tab, tab.data(), tab.size() * 8, s);
  if (e) return e;
  return scalar_mac_dev(c, out, in, k, d_tab, o_c, level, 1, 0, s);
}

// Ragged rotation batch from host job descriptions (each job its own level,
// input, output, key and Galois element; identity jobs copy).
int rotate_jobs(he_ctx* c, std::vector<KsJob>& jobs, int epi, Arena& ar, hipStream_t s) {
  const int n = c->n;
  const int count = (int)jobs.size();
  int lmax = 1;
  for (auto& j : jobs) lmax = std::max(lmax, j.level);
  const int pg = p_groups(c, lmax);
  const int chunk = chunk_for(ar, count, lmax, pg, n);
  if (chunk < 1) return fail(c, HE_ENOMEM, "workspace too small for a batched rotation");
  Arena sub = ar;
  KsScratch ks;
  if (!take_scratch(sub, chunk, lmax, pg, n, ks)) return fail(c, HE_ENOMEM, "workspace too small");
  for (int b0 = 0; b0 < count; b0 += chunk) {
    const int cn = std::min(chunk, count - b0);
    int e = upload(c, ks.jobs, jobs.data() + b0, (size_t)cn * sizeof(KsJob), s);
    if (e) return e;
    bool any_key = false;
    for (int b = b0; b < b0 + cn; ++b) any_key |= jobs[b].key != nullptr;
    if (any_key)
      dispatch_logn<LKsCore>(c->logn, c, (const KsJob*)ks.jobs, cn, lmax, pg, ks.dcoef, ks.u, ks.rc, s);
    dispatch_logn<LDrop>(c->logn, c, (int)MODE_P, epi, (const KsJob*)ks.jobs, cn, lmax, lmax + pg,
                         (const u64*)ks.u, (const u64*)ks.rc, s);
  }
  return check_launch(c, "batched rotation");
}

// Workspace bytes of an FFConv run over n_layers layers (layer buffers plus
// the DensePack chunk temporaries at the largest chunk).
size_t ffconv_need(const he_ctx* c, int n_layers, int level, int spatial, int r, int o_c2, bool square) {
  auto al = [](size_t elems) { return ((elems * 8 + 255) & ~(size_t)255); };
  const size_t n = c->n;
  const int l1 = level - 1, l2 = level - 2;
  const size_t total = (size_t)n_layers * r * spatial;
  size_t need = al(total * 2 * l1 * n) + al((size_t)n_layers * r * 2 * l1 * n) +
                al((size_t)n_layers * o_c2 * 2 * l1 * n) + (square ? 2 * al((size_t)n_layers * o_c2 * 2 * l2 * n) : 0);
  const size_t chunk = std::min<size_t>(total, 16000);
  const int pg = p_groups(c, level);
  need += al(chunk * 2 * level * n) + chunk * 8 * (ks_elems_per_job(level, pg, n) + 2 * (size_t)n + 128 + 256);
  return need + ((size_t)64 << 20);
}

int ffconv_tail(he_ctx* c, int n_layers, const u64* y, int l1, int spatial, int r, const u64* d_mask,
                const u64* d_w2tab, int o_c2, int square, u64* d_out, Arena& ar, hipStream_t s,
                bool shared_w2 = false);

// FFConv over n_layers independent layers of one geometry (layer l: input at
// d_in + l in_stride, W1 base filters at d_w1 + l f_stride, W2 integer table
// at d_w2tab + l 2 r o_c2 (level - 1)): W1 DensePack, DP->CP gather with the
// one-hot mask, 1x1 ConvPack with exact integer weights, rescale, optional
// square + relinearise + rescale.  Outputs d_out [n_layers][o_c2][2][..][N].
int ffconv_run(he_ctx* c, int n_layers, const u64* d_in, size_t in_stride, int level, const he_conv_desc* desc,
               const u64* d_w1, size_t f_stride, const u64* d_mask, const u64* d_w2tab, int o_c2, int square,
               u64* d_out, Arena& ar, hipStream_t s) {
  const int need = square ? 4 : 3;
  if (level < need || level > c->big_l) return fail(c, HE_ELEVEL, "ffconv needs level >= %d (got %d)", need, level);
  c->counts = he_counts{};
  DPGeom geo;
  int n_cls = 0;
  if (!build_geom(c, desc, geo, n_cls)) return fail(c, HE_EINVAL, "bad convolution geometry");
  const int n = c->n;
  const int r = desc->o_c;
  const int spatial = geo.out_h * geo.out_w;
  const int l1 = level - 1;
  if ((long long)n_layers * r > 65535 || (long long)n_layers * o_c2 > 65535)
    return fail(c, HE_EINVAL, "too many layers for one call");
  const size_t B = (size_t)n_layers;
  u64* y = ar.take<u64>(B * r * spatial * 2 * l1 * n);
  if (!y) return fail(c, HE_ENOMEM, "workspace too small for the FFConv layer");
  // 1. W1 under DensePack (HMA, rotate-and-sum, rescale), all layers in one batch
  int e = densepack_run(c, d_in, level, desc, d_w1, y, ar, s, n_layers, in_stride, f_stride);
  if (e) return e;
  return ffconv_tail(c, n_layers, y, l1, spatial, r, d_mask, d_w2tab, o_c2, square, d_out, ar, s);
}

// Steps 2-5 of ffconv_run from the rescaled W1 DensePack outputs y
// ([n_layers][r][S][2][l1][N]): gather, 1x1 ConvPack, rescale, optional
// square + relinearise + rescale.  shared_w2: every layer uses the one
// table at d_w2tab.
int ffconv_tail(he_ctx* c, int n_layers, const u64* y, int l1, int spatial, int r, const u64* d_mask,
                const u64* d_w2tab, int o_c2, int square, u64* d_out, Arena& ar, hipStream_t s, bool shared_w2) {
  const int n = c->n;
  const int l2 = l1 - 1;
  const size_t B = (size_t)n_layers;
  u64* g = ar.take<u64>(B * r * 2 * l1 * n);
  u64* z = ar.take<u64>(B * o_c2 * 2 * l1 * n);
  u64* zr = square ? ar.take<u64>(B * o_c2 * 2 * l2 * n) : nullptr;
  u64* sq = square ? ar.take<u64>(B * o_c2 * 2 * l2 * n) : nullptr;
  if (!g || !z || (square && (!zr || !sq))) return fail(c, HE_ENOMEM, "workspace too small for the FFConv layer");
  int e = HE_OK;
  // 2. DP->CP gather: G_c = sum_p y_{c,p} * sigma_{5^-p}(E), one accumulator per (layer, c)
  const u32 g5inv = galois_of(-1, n);  // 5^-1 in the group of odd residues mod 2N
  dispatch_logn<LHmaPerm>(c->logn, c, g, (const u64*)y, spatial, d_mask, 0, l1, (const int32_t*)nullptr, g5inv, l1, 0,
                          n_layers * r, s);
  if ((e = check_launch(c, "gather"))) return e;
  // 3. 1x1 ConvPack with exact integer weights round(W2 * 2^k)
  if ((e = scalar_mac_dev(c, z, g, r, d_w2tab, o_c2, l1, n_layers, (size_t)r * 2 * l1 * n, s, shared_w2))) return e;
  // 4. rescale; 5. optional square + relinearise + rescale
  const int nz = n_layers * o_c2;
  if (!square) {
    e = rescale_batch(c, d_out, z, nz, l1, ar, s);
  } else {
    e = rescale_batch(c, zr, z, nz, l1, ar, s);
    if (!e) e = square_batch(c, sq, zr, nz, l2, ar, s);
    if (!e) e = rescale_batch(c, d_out, sq, nz, l2, ar, s);
  }
  c->counts.mulpc += (int64_t)n_layers * r * spatial;  // gather masks
  c->counts.addcc += (int64_t)n_layers * (r * (spatial - 1) + o_c2 * (r - 1));
  c->counts.scalar_mul += (int64_t)n_layers * r * o_c2;
  c->counts.rescale += (int64_t)nz * (square ? 2 : 1);
  c->counts.square += square ? nz : 0;
  return e;
}

// Inner products, P INTT and ModDown of m hoisted rotations whose
// inner-product rows (u) and P-limb coefficients (rc) all fit: the rows of
// chunk k are computed on s while chunk k - 1 is taken down on the side
// stream (the first stage streams keys from HBM, the second is transform
// arithmetic), then s waits for the side stream.  Without a side stream or
// with few rotations, one stream.
void hoisted_rest(he_ctx* c, const KsJob* jobs, int m, int level, const u64* dhat, u64* u, u64* rc, hipStream_t s,
                  int per_ct, size_t dstride) {
  const int n = c->n;
  const int sub = m >= 64 ? (m + 3) / 4 : m;  // at most 4 chunks: one event each
  if (!c->side || !c->hoist_pipeline || sub == m) {
    dispatch_logn<LHoisted>(c->logn, c, jobs, m, level, dhat, u, rc, s, 0, per_ct, dstride);
    return;
  }
  for (int r0 = 0, k = 0; r0 < m; r0 += sub, ++k) {
    const int cm = std::min(sub, m - r0);
    u64* ur = u + (size_t)r0 * 2 * (level + 1) * n;
    u64* rr = rc + (size_t)r0 * 2 * n;
    dispatch_logn<LHoisted>(c->logn, c, jobs + r0, cm, level, dhat, ur, rr, s, r0, per_ct, dstride, 1);
    // the side stream sees everything s did up to this chunk's inner products
    (void)hipEventRecord(c->pipe_ev[k], s);
    (void)hipStreamWaitEvent(c->side, c->pipe_ev[k], 0);
    dispatch_logn<LHoisted>(c->logn, c, jobs + r0, cm, level, dhat, ur, rr, c->side, r0, per_ct, dstride, 2);
  }
  (void)hipEventRecord(c->join_ev, c->side);
  (void)hipStreamWaitEvent(s, c->join_ev, 0);
}

// Rotations of n_in ciphertexts (ciphertext i at in + i in_stride,
// [2][level][N]) by the m rotations of hk; the rotations of one ciphertext
// share its digit decomposition and ModUp.  out = [n_in][m][2][level][N]
// (with out_stride: rotation r of ciphertext i at out + i out_stride +
// r 2 level N).
// Ciphertexts go in passes that fit the workspace (a single ciphertext's
// rotations in chunks when even one does not fit whole).
int hoisted_batch(he_ctx* c, const u64* in, size_t in_stride, int n_in, int level, const HoistKeys& hk, int m,
                  u64* out, Arena& ar, hipStream_t s, size_t out_stride = 0) {
  const int n = c->n;
  const size_t per_ct = (size_t)level * n + (size_t)level * (level + 1) * n + 128;  // digits, lifted digits
  const size_t per_rot = (size_t)2 * (level + 2) * n + 64;                         // u rows, ModDown input, job
  const size_t left = ar.left() / 8;
  size_t cc = std::min<size_t>({(size_t)n_in, (size_t)(32000 / m), left / (per_ct + (size_t)m * per_rot)});
  size_t rch = cc * m;
  if (cc < 1) {
    cc = 1;
    if (left < per_ct + (size_t)m * 8 + per_rot + 256)
      return fail(c, HE_ENOMEM, "workspace too small for hoisted rotations at level %d", level);
    rch = std::min<size_t>(m, (left - per_ct - (size_t)m * 8 - 256) / per_rot);
  }
  Arena sub = ar;
  KsJob* jobs1 = sub.take<KsJob>(cc);
  KsJob* jobs = sub.take<KsJob>(cc * m);
  u64* dcoef = sub.take<u64>(cc * level * n);
  u64* dhat = sub.take<u64>(cc * level * (level + 1) * n);
  u64* u = sub.take<u64>(rch * 2 * (level + 1) * n);
  u64* rc = sub.take<u64>(rch * 2 * n);
  if (!jobs1 || !jobs || !dcoef || !dhat || !u || !rc)
    return fail(c, HE_ENOMEM, "workspace too small for hoisted rotations at level %d", level);
  const size_t ostride = out_stride ? out_stride : (size_t)m * 2 * level * n;  // between input ciphertexts
  for (int i0 = 0; i0 < n_in; i0 += (int)cc) {
    const int cn = std::min((int)cc, n_in - i0);
    const u64* cin = in + (size_t)i0 * in_stride;
    u64* cout = out + (size_t)i0 * ostride;
    k_make_hoist_jobs<<<dim3((cn + 255) / 256, 1), 256, 0, s>>>(jobs1, cn, 1, cin, in_stride, cout, ostride, level, n,
                                                                 hk, 1);
    k_make_hoist_jobs<<<dim3((cn + 255) / 256, m), 256, 0, s>>>(jobs, cn, m, cin, in_stride, cout, ostride, level, n,
                                                                 hk, 0);
    dispatch_logn<LHoistUp>(c->logn, c, (const KsJob*)jobs1, cn, level, dcoef, dhat, s);
    const int total = cn * m;
    if ((int)rch >= total) {
      hoisted_rest(c, jobs, total, level, dhat, u, rc, s, m, (size_t)level * (level + 1) * n);
      continue;
    }
    for (int r0 = 0; r0 < total; r0 += (int)rch) {
      const int cm = std::min((int)rch, total - r0);
      dispatch_logn<LHoisted>(c->logn, c, (const KsJob*)(jobs + r0), cm, level, (const u64*)dhat, u, rc, s, r0, m,
                              (size_t)level * (level + 1) * n);
    }
  }
  return check_launch(c, "hoisted rotations");
}

// Key inner products (over Q and P, with P sigma_g(c0) added to u_0) of n_in
// ciphertexts' hoisted rotations, no ModDown: u = [n_in][m][2][level + 1][N]
// in the key-switch row layout (narrow rows packed), all of it the caller's.
int hoisted_ip(he_ctx* c, const u64* in, size_t in_stride, int n_in, int level, const HoistKeys& hk, int m, u64* u,
               Arena& ar, hipStream_t s) {
  const int n = c->n;
  const size_t per_ct = (size_t)level * n + (size_t)level * (level + 1) * n + 128 + (size_t)m * 8;
  const size_t cc = std::min<size_t>({(size_t)n_in, (size_t)(32000 / m), ar.left() / 8 / per_ct});
  if (cc < 1) return fail(c, HE_ENOMEM, "workspace too small for hoisted inner products at level %d", level);
  Arena sub = ar;
  KsJob* jobs1 = sub.take<KsJob>(cc);
  KsJob* jobs = sub.take<KsJob>(cc * m);
  u64* dcoef = sub.take<u64>(cc * level * n);
  u64* dhat = sub.take<u64>(cc * level * (level + 1) * n);
  if (!jobs1 || !jobs || !dcoef || !dhat) return fail(c, HE_ENOMEM, "workspace too small for hoisted inner products");
  const size_t ustride = (size_t)m * 2 * (level + 1) * n;  // per input ciphertext
  for (int i0 = 0; i0 < n_in; i0 += (int)cc) {
    const int cn = std::min((int)cc, n_in - i0);
    const u64* cin = in + (size_t)i0 * in_stride;
    u64* ui = u + (size_t)i0 * ustride;
    k_make_hoist_jobs<<<dim3((cn + 255) / 256, 1), 256, 0, s>>>(jobs1, cn, 1, cin, in_stride, ui, ustride, level, n,
                                                                 hk, 1);
    k_make_hoist_jobs<<<dim3((cn + 255) / 256, m), 256, 0, s>>>(jobs, cn, m, cin, in_stride, ui, ustride, level, n,
                                                                 hk, 0);
    dispatch_logn<LHoistUp>(c->logn, c, (const KsJob*)jobs1, cn, level, dcoef, dhat, s);
    dispatch_logn<LHoisted>(c->logn, c, (const KsJob*)jobs, cn * m, level, (const u64*)dhat, ui, (u64*)nullptr, s, 0,
                            m, (size_t)level * (level + 1) * n, 1, 1);
  }
  return check_launch(c, "hoisted inner products");
}

// ---- Tap-style DensePack ------------------------------------------------------
// Input in the DensePack layout (channel c of ciphertext m in block
// b = c - m B at slots b H W + h W + w); each ciphertext is rotated by the
// d^2 tap shifts (kh - pad) W + (kw - pad), hoisted; the masked weight
// plaintexts F[o][m][t] multiply and sum them; the blocks are summed into
// block 0 by the binary schedule; one rescale.  Output (i, j) of channel o
// at slot (s i) W + s j.

struct TapPlan {
  int per = 0, m_cts = 0, hw = 0, nrot = 0;
  TapMap map{};
  HoistKeys hk{};
  std::vector<std::pair<int, int>> sched;  // (0: S + Rot(S, a), 1: t + Rot(S, a); a = rotation)
  bool has_inc = false;
};

// need_keys false: the geometry only (for workspace sizes).
int tap_plan(he_ctx* c, const char* who, const he_conv_desc* g, TapPlan& tp, bool need_keys = true) {
  const int slots = c->n / 2;
  if (g->h < 1 || g->w < 1 || g->c_in < 1 || g->d < 1 || g->stride < 1 || g->pad < 0 || 2 * g->pad > g->d - 1 ||
      g->d > g->h || g->d > g->w || g->d * g->d > 64 || g->o_c < 1 || g->o_c > 65535 ||
      (long long)g->h * g->w > slots)
    return fail(c, HE_EINVAL, "%s: unsupported geometry (%dx%dx%d, d %d, stride %d, pad %d)", who, g->h, g->w, g->c_in,
                g->d, g->stride, g->pad);
  const int n = c->n;
  tp.hw = g->h * g->w;
  tp.per = std::min(slots / tp.hw, g->c_in);
  tp.m_cts = (g->c_in + tp.per - 1) / tp.per;
  const int d2 = g->d * g->d;
  tp.nrot = 0;
  for (int t = 0; t < d2; ++t) {
    const int kh = t / g->d, kw = t % g->d;
    int sh = ((kh - g->pad) * g->w + (kw - g->pad)) % slots;
    if (sh < 0) sh += slots;
    if (sh == 0) {
      tp.map.idx[t] = -1;
      continue;
    }
    const u32 gal = galois_of(sh, n);
    auto it = c->keys.find((int)gal);
    if (need_keys && it == c->keys.end()) return fail(c, HE_ENOKEY, "%s: no rotation key for tap shift %d", who, sh);
    tp.hk.key[tp.nrot] = it == c->keys.end() ? nullptr : it->second;
    tp.hk.g[tp.nrot] = gal;
    tp.hk.ginv[tp.nrot] = galois_of(-sh, n);
    tp.map.idx[t] = (signed char)tp.nrot;
    ++tp.nrot;
  }
  tp.map.d2 = d2;
  tp.map.m_cts = tp.m_cts;
  tp.map.o_c = g->o_c;
  tp.map.nrot = tp.nrot;
  tp.sched.clear();
  tp.has_inc = false;
  int k = 1, top = 0;
  while ((tp.per >> (top + 1)) != 0) ++top;
  for (int bit = top - 1; bit >= 0; --bit) {
    tp.sched.push_back({0, k * tp.hw});
    k *= 2;
    if ((tp.per >> bit) & 1) {
      tp.sched.push_back({1, tp.hw});
      tp.has_inc = true;
      k += 1;
    }
  }
  for (auto& st : tp.sched)
    if (need_keys && !c->keys.count((int)galois_of(st.second, n)))
      return fail(c, HE_ENOKEY, "%s: no rotation key for block step %d", who, st.second);
  return HE_OK;
}

size_t tap_need(const he_ctx* c, const TapPlan& tp, int nb, int level) {
  auto al = [](size_t elems) { return ((elems * 8 + 255) & ~(size_t)255); };
  const size_t n = c->n, cs = 2 * (size_t)level * n, us = 2 * (size_t)(level + 1) * n;
  const size_t o = (size_t)nb * tp.map.o_c;
  // rotated ciphertexts, or with a deferred ModDown their inner-product rows and the outputs' rows
  size_t need = std::max(al((size_t)nb * tp.m_cts * tp.nrot * cs),
                         al((size_t)nb * tp.m_cts * tp.nrot * us) + al(o * us) + al(o * 2 * n) + al(o * 8)) +
                al(o * cs) * (tp.has_inc ? 2 : 1);
  // one ciphertext's hoisting with all its rotations, and a key-switch chunk of the block sum
  const size_t hoist = ((size_t)level * n + (size_t)level * (level + 1) * n + 128 +
                        (size_t)tp.nrot * (2 * (level + 2) * n + 64)) * 8 + 4096;
  const size_t ks = std::min<size_t>(o, 4096) * 8 *
                    (ks_elems_per_job(level, p_groups(const_cast<he_ctx*>(c), level), (int)n) + 128);
  return need + std::max(hoist, ks) + ((size_t)16 << 20);
}

// out = [nb][O][2][level - 1][N] from in = [nb][M][2][level][N]; filt =
// [O][M][d^2][pt_limbs][N]; filt_p (or null) the same plaintexts mod P,
// [O][M][d^2][N]: with it one ModDown per output after the products over
// (Q, P), else one per rotation before them.  Adds its counts.
int tap_run(he_ctx* c, const TapPlan& tp, int nb, const u64* in, int level, const u64* filt, int pt_limbs,
            const u64* filt_p, u64* out, Arena& ar, hipStream_t s) {
  const int n = c->n;
  const int o_c = tp.map.o_c;
  const size_t cs = (size_t)2 * level * n;
  const int n_in = nb * tp.m_cts;
  const int n_out = nb * o_c;
  const bool lazy = filt_p != nullptr && tp.nrot > 0;
  const size_t us = (size_t)2 * (level + 1) * n;
  u64* t = ar.take<u64>((size_t)n_out * cs);
  u64* t0 = tp.has_inc ? ar.take<u64>((size_t)n_out * cs) : nullptr;
  if (!t || (tp.has_inc && !t0)) return fail(c, HE_ENOMEM, "workspace too small for the tap-style layer");
  int e = HE_OK;
  if (lazy) {
    Arena la = ar;  // the rows below are free once the ModDown has run
    u64* uq = la.take<u64>((size_t)n_in * tp.nrot * us);
    u64* uo = la.take<u64>((size_t)n_out * us);
    u64* rc = la.take<u64>((size_t)n_out * 2 * n);
    KsJob* dj = la.take<KsJob>(n_out);
    if (!uq || !uo || !rc || !dj) return fail(c, HE_ENOMEM, "workspace too small for the tap-style layer");
    if ((e = hoisted_ip(c, in, cs, n_in, level, tp.hk, tp.nrot, uq, la, s))) return e;
    dispatch_logn<LTapHmaQp>(c->logn, c, in, (const u64*)uq, filt, filt_p, uo, level, pt_limbs, tp.map, nb, s);
    make_jobs(c, dj, n_out, t, cs, t, cs, t, cs, tp.hk.key[0], 1u, 1u, level, s);
    dispatch_logn<LModDown>(c->logn, c, (const KsJob*)dj, n_out, level, (const u64*)uo, rc, s);
    if ((e = check_launch(c, "tap_hma_qp"))) return e;
  } else {
    u64* rot = tp.nrot ? ar.take<u64>((size_t)n_in * tp.nrot * cs) : nullptr;
    if (tp.nrot && !rot) return fail(c, HE_ENOMEM, "workspace too small for the tap-style layer");
    if (tp.nrot && (e = hoisted_batch(c, in, cs, n_in, level, tp.hk, tp.nrot, rot, ar, s))) return e;
    dispatch_logn<LTapHma>(c->logn, c, in, (const u64*)rot, filt, t, level, pt_limbs, tp.map, nb, s);
    if ((e = check_launch(c, "tap_hma"))) return e;
  }
  if (tp.has_inc && hipMemcpyAsync(t0, t, (size_t)n_out * cs * 8, hipMemcpyDeviceToDevice, s) != hipSuccess)
    return fail(c, HE_EDEVICE, "tap-style layer: device copy failed");
  for (auto& st : tp.sched) {
    e = rotate_batch(c, t, t, n_out, level, st.second, st.first == 0 ? EPI_ROTSUM : EPI_ROT, ar, s);
    if (!e && st.first == 1) {
      k_add<<<dim3(n / 256, level, n_out), 256, 0, s>>>(t, t0, t, level, n, c->mods);
      e = check_launch(c, "tap-style block sum");
    }
    if (e) return e;
  }
  if ((e = rescale_batch(c, out, t, n_out, level, ar, s))) return e;
  const int64_t d2 = tp.map.d2, steps = (int64_t)tp.sched.size();
  c->counts.rot += (int64_t)n_in * tp.nrot + (int64_t)n_out * steps;
  c->counts.mulpc += (int64_t)n_out * tp.m_cts * d2;
  c->counts.addcc += (int64_t)n_out * (tp.m_cts * d2 - 1 + steps);
  c->counts.rescale += n_out;
  return HE_OK;
}

// ---- Homomorphic Im2Col (d > 1) ---------------------------------------------
struct Him2colPlan {
  int per = 0, m_cts = 0, hw = 0, nrot = 0, last = 0;  // last: channels in the last input ciphertext
  Him2colMap map{};
  HoistKeys tap{}, blk{};
  int nblk = 0;
};

int him2col_plan(he_ctx* c, const he_conv_desc* g, Him2colPlan& hp, bool need_keys = true) {
  TapPlan tp;
  he_conv_desc d1 = *g;
  d1.o_c = 1;
  int e = tap_plan(c, "he_him2col", &d1, tp, false);
  if (e) return e;
  const int n = c->n;
  hp.per = tp.per;
  hp.m_cts = tp.m_cts;
  hp.hw = tp.hw;
  hp.nrot = tp.nrot;
  hp.tap = tp.hk;
  hp.last = g->c_in - (tp.m_cts - 1) * tp.per;
  hp.nblk = tp.per - 1;
  if (hp.nblk > MAX_HOIST) return fail(c, HE_EINVAL, "he_him2col: %d channels per ciphertext (at most %d)", tp.per,
                                       MAX_HOIST + 1);
  for (int r = 0; r < tp.nrot; ++r)
    if (need_keys && !tp.hk.key[r]) return fail(c, HE_ENOKEY, "he_him2col: no rotation key for a tap shift");
  for (int b = 1; b < tp.per; ++b) {
    const u32 gal = galois_of(b * tp.hw, n);
    auto it = c->keys.find((int)gal);
    if (need_keys && it == c->keys.end()) return fail(c, HE_ENOKEY, "he_him2col: no rotation key for block shift %d",
                                                      b * tp.hw);
    hp.blk.key[b - 1] = it == c->keys.end() ? nullptr : it->second;
    hp.blk.g[b - 1] = gal;
    hp.blk.ginv[b - 1] = galois_of(-b * tp.hw, n);
  }
  hp.map.d2 = g->d * g->d;
  hp.map.c_in = g->c_in;
  hp.map.per = tp.per;
  hp.map.m_cts = tp.m_cts;
  hp.map.nrot = tp.nrot;
  hp.map.nvalid = g->c_in;  // (M - 1) B + last
  for (int t = 0; t < hp.map.d2; ++t) hp.map.idx[t] = tp.map.idx[t];
  return HE_OK;
}

size_t him2col_need(const he_ctx* c, const Him2colPlan& hp, int nb, int level) {
  auto al = [](size_t elems) { return ((elems * 8 + 255) & ~(size_t)255); };
  const size_t n = c->n, cs = 2 * (size_t)level * n;
  const size_t k = (size_t)hp.map.d2 * hp.map.c_in;
  size_t need = al((size_t)nb * hp.m_cts * hp.per * cs) + al((size_t)nb * hp.map.nvalid * hp.nrot * cs) +
                al((size_t)nb * k * cs);
  const int m = std::max(1, std::max(hp.nrot, hp.nblk));
  need += ((size_t)level * n + (size_t)level * (level + 1) * n + 128 + (size_t)m * (2 * (level + 2) * n + 64)) * 8 +
          std::min<size_t>((size_t)nb * k, 32000) * (2 * n + 64) * 8;
  return need + ((size_t)16 << 20);
}

}  // namespace

// =============================================================================
// Public entry points
// =============================================================================

extern "C" {

int he_params_moduli(const he_params* p, uint64_t* h_out) {
  if (!p || !h_out) return HE_EINVAL;
  return gen_moduli(p->n, p->n_q, p->q_bits, p->p_bits, h_out) ? HE_EINVAL : HE_OK;
}

int he_ctx_create(const he_params* p, he_ctx** out) {
  if (!p || !out) return HE_EINVAL;
  *out = nullptr;
  int logn = 0;
  while ((1 << logn) < p->n) ++logn;
  if ((1 << logn) != p->n || logn < 10 || logn > 14) return HE_EUNSUPPORTED;
  if (p->n_q < 1 || p->n_q >= HE_MAXM) return HE_EINVAL;
  std::vector<u64> mods(p->n_q + 1);
  if (gen_moduli(p->n, p->n_q, p->q_bits, p->p_bits, mods.data())) return HE_EINVAL;
  he_ctx* c = new he_ctx();
  c->n = p->n;
  c->logn = logn;
  c->big_l = p->n_q;
  c->moduli = mods;
  (void)hipGetDevice(&c->device);
  for (int i = 0; i <= p->n_q; ++i) {
    c->mods.m[i] = make_modconst(mods[i], p->n);
    c->has_cls[c->mods.m[i].cls] = true;
    if (i < p->n_q) c->q_mask |= 1u << c->mods.m[i].cls;
  }
  c->p_cls = (int)c->mods.m[p->n_q].cls;
  const size_t n = p->n;
  std::vector<u64> tw(mods.size() * 4 * n);
  for (size_t i = 0; i < mods.size(); ++i) {
    u64* b = tw.data() + i * 4 * n;
    make_twiddles(mods[i], p->n, b, b + n, b + 2 * n, b + 3 * n);
  }
  std::vector<u32> tw32(tw.size(), 0);
  std::vector<double> twf(tw.size(), 0.0);
  for (size_t i = 0; i < mods.size(); ++i) {
    const u64* b = tw.data() + i * 4 * n;
    if (is_narrow(mods[i]))
      for (size_t k = 0; k < 4 * n; ++k) tw32[i * 4 * n + k] = (u32)b[k];
    if (width_class(mods[i]) == CLS_F64)
      for (size_t k = 0; k < n; ++k) {  // (w, w / q) for the forward and inverse tables
        double* f = twf.data() + i * 4 * n;
        f[k] = (double)b[k];
        f[n + k] = (double)b[k] / (double)mods[i];
        f[2 * n + k] = (double)b[2 * n + k];
        f[3 * n + k] = (double)b[2 * n + k] / (double)mods[i];
      }
  }
  // Half-ring forward twiddles: after the first stage (pairs i, i + N/2 with
  // w[1]) the two halves are independent transforms of N/2 points; stage s'
  // of half h uses, for block k' < 2^s', the full table's w[2^(s'+1) + h 2^s'
  // + k'], stored at index 2^s' + k' of that half's table.
  const size_t nh = n / 2;
  std::vector<u64> twh(mods.size() * 4 * nh, 0);
  for (size_t i = 0; i < mods.size(); ++i)
    for (int h = 0; h < 2; ++h) {
      const u64* fw = tw.data() + i * 4 * n;
      u64* dst = twh.data() + (i * 2 + h) * 2 * nh;
      for (size_t mp = 1; mp < nh; mp <<= 1)
        for (size_t k = 0; k < mp; ++k) {
          dst[mp + k] = fw[2 * mp + h * mp + k];
          dst[nh + mp + k] = fw[n + 2 * mp + h * mp + k];
        }
    }
  std::vector<u32> twh32(twh.size(), 0);
  std::vector<double> twhf(twh.size(), 0.0);
  for (size_t i = 0; i < mods.size(); ++i) {
    const size_t o = i * 4 * nh;
    if (is_narrow(mods[i]))
      for (size_t k = 0; k < 4 * nh; ++k) twh32[o + k] = (u32)twh[o + k];
    if (width_class(mods[i]) == CLS_F64)
      for (size_t k = 0; k < 4 * nh; ++k) twhf[o + k] = (double)twh[o + k];
  }
  // inverse table: inv[div][t] = m_div^-1 mod q_t for divisors 0..L (L = P)
  std::vector<u64> inv(2 * HE_MAXM * HE_MAXM, 0);
  for (int dv = 0; dv <= p->n_q; ++dv)
    for (int t = 0; t < p->n_q; ++t) {
      if (t == dv) continue;
      const u64 v = inv_mod(mods[dv] % mods[t], mods[t]);
      inv[dv * HE_MAXM + t] = v;
      inv[HE_MAXM * HE_MAXM + dv * HE_MAXM + t] = shoup_companion(v, mods[t]);
    }
  bool ok = hipMalloc((void**)&c->d_tw, tw.size() * 8) == hipSuccess &&
                  hipMemcpy(c->d_tw, tw.data(), tw.size() * 8, hipMemcpyHostToDevice) == hipSuccess &&
                  hipMalloc((void**)&c->d_tw32, tw32.size() * 4) == hipSuccess &&
                  hipMemcpy(c->d_tw32, tw32.data(), tw32.size() * 4, hipMemcpyHostToDevice) == hipSuccess &&
                  hipMalloc((void**)&c->d_twf, twf.size() * 8) == hipSuccess &&
                  hipMemcpy(c->d_twf, twf.data(), twf.size() * 8, hipMemcpyHostToDevice) == hipSuccess &&
                  hipMalloc((void**)&c->d_twh, twh.size() * 8) == hipSuccess &&
                  hipMemcpy(c->d_twh, twh.data(), twh.size() * 8, hipMemcpyHostToDevice) == hipSuccess &&
                  hipMalloc((void**)&c->d_twh32, twh32.size() * 4) == hipSuccess &&
                  hipMemcpy(c->d_twh32, twh32.data(), twh32.size() * 4, hipMemcpyHostToDevice) == hipSuccess &&
                  hipMalloc((void**)&c->d_twhf, twhf.size() * 8) == hipSuccess &&
                  hipMemcpy(c->d_twhf, twhf.data(), twhf.size() * 8, hipMemcpyHostToDevice) == hipSuccess &&
                  hipMalloc((void**)&c->d_inv, inv.size() * 8) == hipSuccess &&
                  hipMemcpy(c->d_inv, inv.data(), inv.size() * 8, hipMemcpyHostToDevice) == hipSuccess &&
                  hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking) == hipSuccess &&
                  hipEventCreateWithFlags(&c->fork_ev, hipEventDisableTiming) == hipSuccess &&
                  hipEventCreateWithFlags(&c->join_ev, hipEventDisableTiming) == hipSuccess &&
                  hipEventCreateWithFlags(&c->pipe_ev[0], hipEventDisableTiming) == hipSuccess &&
                  hipEventCreateWithFlags(&c->pipe_ev[1], hipEventDisableTiming) == hipSuccess &&
                  hipEventCreateWithFlags(&c->pipe_ev[2], hipEventDisableTiming) == hipSuccess &&
                  hipEventCreateWithFlags(&c->pipe_ev[3], hipEventDisableTiming) == hipSuccess;
  for (int i = 0; ok && i < MAX_SPLIT - 2; ++i)
    ok = hipStreamCreateWithFlags(&c->side_x[i], hipStreamNonBlocking) == hipSuccess &&
         hipEventCreateWithFlags(&c->join_x[i], hipEventDisableTiming) == hipSuccess;
  if (!ok || scratch_setup(c) != HE_OK) {
    he_ctx_destroy(c);
    return HE_EDEVICE;
  }
  *out = c;
  return HE_OK;
}

int he_ctx_destroy(he_ctx* c) {
  if (!c) return HE_EINVAL;
  (void)hipDeviceSynchronize();
  for (auto& pr : c->prof_events) c->prof_pool.insert(c->prof_pool.end(), {pr.first, pr.second});
  for (hipEvent_t e : c->prof_pool) (void)hipEventDestroy(e);
  for (auto& kv : c->keys) (void)hipFree(kv.second);
  (void)hipFree(c->d_tw);
  (void)hipFree(c->d_tw32);
  (void)hipFree(c->d_twf);
  (void)hipFree(c->d_twh);
  (void)hipFree(c->d_twh32);
  (void)hipFree(c->d_twhf);
  (void)hipFree(c->d_inv);
  if (c->ws_owned) (void)hipFree(c->ws);
  if (c->side) (void)hipStreamDestroy(c->side);
  for (int i = 0; i < MAX_SPLIT - 2; ++i) {
    if (c->side_x[i]) (void)hipStreamDestroy(c->side_x[i]);
    if (c->join_x[i]) (void)hipEventDestroy(c->join_x[i]);
  }
  for (hipEvent_t e : c->pipe_ev)
    if (e) (void)hipEventDestroy(e);
  if (c->fork_ev) (void)hipEventDestroy(c->fork_ev);
  if (c->join_ev) (void)hipEventDestroy(c->join_ev);
  for (auto& st : c->stage) {
    if (st.host) (void)hipHostFree(st.host);
    if (st.ev) (void)hipEventDestroy(st.ev);
  }
  delete c;
  return HE_OK;
}

int he_ctx_reserve(he_ctx* c, size_t bytes) {
  if (!c) return HE_EINVAL;
  if (bytes <= c->ws_bytes) return HE_OK;
  if (c->capturing) return fail(c, HE_EUNSUPPORTED, "he_ctx_reserve: not allowed during graph capture");
  ++c->epoch;
  (void)hipDeviceSynchronize();
  if (c->ws_owned) (void)hipFree(c->ws);
  c->ws = nullptr;
  c->ws_bytes = 0;
  c->ws_owned = true;
  if (hipMalloc((void**)&c->ws, bytes) != hipSuccess)
    return fail(c, HE_ENOMEM, "workspace allocation of %zu bytes failed", bytes);
  c->ws_bytes = bytes;
  return HE_OK;
}

int he_ctx_set_workspace(he_ctx* c, void* d_ws, size_t bytes) {
  if (!c || (!d_ws && bytes)) return fail(c, HE_EINVAL, "he_ctx_set_workspace: bad arguments");
  if (((uintptr_t)d_ws & 255) != 0) return fail(c, HE_EINVAL, "he_ctx_set_workspace: buffer not 256-byte aligned");
  if (c->capturing) return fail(c, HE_EUNSUPPORTED, "he_ctx_set_workspace: not allowed during graph capture");
  ++c->epoch;
  (void)hipDeviceSynchronize();
  if (c->ws_owned) (void)hipFree(c->ws);
  c->ws = (char*)d_ws;
  c->ws_bytes = d_ws ? bytes : 0;
  c->ws_owned = false;
  return HE_OK;
}

size_t he_ctx_workspace_need(const he_ctx* c, int count, int level) {
  if (!c || count < 1 || level < 1) return 0;
  // accumulators (2 level), a second batch of that size (layer intermediates),
  // key switch temporaries (3 level + 2 pg + 2, pg <= PG_MAX) and tables, in
  // limbs of N.
  const size_t per = (size_t)(4 * level) + (3 * (size_t)level + 2 * PG_MAX + 2) + 2;
  return (size_t)count * per * c->n * 8 + ((size_t)16 << 20);
}

int he_ctx_moduli(const he_ctx* c, uint64_t* h_out) {
  if (!c || !h_out) return HE_EINVAL;
  for (size_t i = 0; i < c->moduli.size(); ++i) h_out[i] = c->moduli[i];
  return HE_OK;
}

const char* he_last_error(const he_ctx* c) { return c ? c->err.c_str() : "null context"; }

int he_ctx_set_tuning(he_ctx* c, const char* knob, int level, int value) {
  if (!c || !knob) return HE_EINVAL;
  if (std::strcmp(knob, "split_streams") == 0) {
    if (value < 0 || value > 1) return fail(c, HE_EINVAL, "he_ctx_set_tuning: split_streams is 0 or 1");
    c->split_streams = value;
    return HE_OK;
  }
  if (std::strcmp(knob, "moddown_halves") == 0) {
    if (value < -1 || value > 1) return fail(c, HE_EINVAL, "he_ctx_set_tuning: moddown_halves is -1, 0 or 1");
    if (value == 1 && c->logn < HALF_MODUP_ANY_LOGN)
      return fail(c, HE_EINVAL, "he_ctx_set_tuning: moddown_halves needs N >= %d", 1 << HALF_MODUP_ANY_LOGN);
    c->moddown_halves = value;
    return HE_OK;
  }
  if (std::strcmp(knob, "split_parts") == 0) {
    if (value < 2 || value > MAX_SPLIT)
      return fail(c, HE_EINVAL, "he_ctx_set_tuning: split_parts is 2..%d", MAX_SPLIT);
    c->split_parts = value;
    return HE_OK;
  }
  if (std::strcmp(knob, "hoist_pipeline") == 0) {
    if (value < 0 || value > 1) return fail(c, HE_EINVAL, "he_ctx_set_tuning: hoist_pipeline is 0 or 1");
    c->hoist_pipeline = value;
    return HE_OK;
  }
  if (std::strcmp(knob, "hoist_fused") == 0) {
    if (value < 0 || value > 1) return fail(c, HE_EINVAL, "he_ctx_set_tuning: hoist_fused is 0 or 1");
    c->hoist_fused = value;
    return HE_OK;
  }
  if (std::strcmp(knob, "modup_halves") == 0) {
    if (value < -1 || value > 1) return fail(c, HE_EINVAL, "he_ctx_set_tuning: modup_halves is -1, 0 or 1");
    if (level < 0 || level > c->big_l) return fail(c, HE_EINVAL, "he_ctx_set_tuning: level %d out of range", level);
    if (value == 1 && c->logn < HALF_MODUP_ANY_LOGN)
      return fail(c, HE_EINVAL, "he_ctx_set_tuning: modup_halves needs N >= %d", 1 << HALF_MODUP_ANY_LOGN);
    for (int lv = (level ? level : 1); lv <= (level ? level : c->big_l); ++lv) c->halves_set[lv] = value;
    return HE_OK;
  }
  if (std::strcmp(knob, "p_groups") != 0) return fail(c, HE_EINVAL, "he_ctx_set_tuning: unknown knob '%s'", knob);
  if (level < 1 || level > c->big_l || value < 0 || value > std::min(level, PG_MAX))
    return fail(c, HE_EINVAL, "he_ctx_set_tuning: p_groups %d out of range at level %d", value, level);
  c->pg_set[level] = value;
  return HE_OK;
}

int he_ctx_get_tuning(const he_ctx* c, const char* knob, int level) {
  if (!c || !knob) return HE_EINVAL;
  if (std::strcmp(knob, "split_streams") == 0) return c->split_streams;
  if (std::strcmp(knob, "split_parts") == 0) return c->split_parts;
  if (std::strcmp(knob, "moddown_halves") == 0)
    return c->moddown_halves < 0 ? (c->logn >= HALF_MODDOWN_MIN_LOGN ? 1 : 0) : c->moddown_halves;
  if (std::strcmp(knob, "hoist_fused") == 0) return c->hoist_fused;
  if (std::strcmp(knob, "hoist_pipeline") == 0) return c->hoist_pipeline;
  if (std::strcmp(knob, "modup_halves") == 0) {
    const int lv = level ? level : c->big_l;
    if (lv < 1 || lv > c->big_l) return HE_EINVAL;
    return c->halves_set[lv] < 0 ? (c->logn >= HALF_MODUP_MIN_LOGN ? 1 : 0) : c->halves_set[lv];
  }
  if (std::strcmp(knob, "p_groups") != 0 || level < 1 || level > c->big_l) return HE_EINVAL;
  return p_groups(c, level);
}

int he_ntt(he_ctx* c, uint64_t* d, int n_polys, int n_limbs, int first_mod, void* stream) {
  if (!c || !d || n_polys < 1 || n_limbs < 1 || n_polys > 65535 || first_mod < 0 || first_mod + n_limbs > c->big_l + 1)
    return fail(c, HE_EINVAL, "he_ntt: bad arguments");
  dispatch_logn<LNtt>(c->logn, c, d, n_polys, n_limbs, first_mod, true, S(stream));
  return check_launch(c, "he_ntt");
}

int he_intt(he_ctx* c, uint64_t* d, int n_polys, int n_limbs, int first_mod, void* stream) {
  if (!c || !d || n_polys < 1 || n_limbs < 1 || n_polys > 65535 || first_mod < 0 || first_mod + n_limbs > c->big_l + 1)
    return fail(c, HE_EINVAL, "he_intt: bad arguments");
  dispatch_logn<LNtt>(c->logn, c, d, n_polys, n_limbs, first_mod, false, S(stream));
  return check_launch(c, "he_intt");
}

int he_add(he_ctx* c, uint64_t* out, const uint64_t* a, const uint64_t* b, int count, int level, double scale_a,
           double scale_b, void* stream) {
  if (!c || !out || !a || !b || count < 1 || count > 65535 || !level_ok(c, level))
    return fail(c, HE_EINVAL, "he_add: bad arguments");
  if (!scales_agree(scale_a, scale_b))
    return fail(c, HE_ESCALE, "he_add: scales %.17g and %.17g differ", scale_a, scale_b);
  Prof pr(c, "add", S(stream));
  k_add<<<dim3(c->n / 256, level, count), 256, 0, S(stream)>>>(out, a, b, level, c->n, c->mods);
  return check_launch(c, "he_add");
}

int he_hma_plain(he_ctx* c, uint64_t* acc, const uint64_t* cts, int k, const uint64_t* pts, int pt_stride, int pt_limbs,
                 const int32_t* h_galois, int level, int accumulate, double ct_scale, double pt_scale,
                 double* io_acc_scale, void* stream) {
  if (!c || !acc || !cts || !pts || !io_acc_scale || k < 1 || pt_stride < 0 || pt_limbs < level || !level_ok(c, level))
    return fail(c, HE_EINVAL, "he_hma_plain: bad arguments");
  const double prod_scale = ct_scale * pt_scale;
  if (!scale_ok(ct_scale) || !scale_ok(pt_scale) || !scale_ok(prod_scale) ||
      (accumulate && !scales_agree(*io_acc_scale, prod_scale)))
    return fail(c, HE_ESCALE, "he_hma_plain: product scale %.17g does not match the accumulator's %.17g", prod_scale,
                *io_acc_scale);
  Arena ar(c);
  const int32_t* d_gal = nullptr;
  if (h_galois) {
    for (int i = 0; i < k; ++i)
      if (h_galois[i] <= 0 || h_galois[i] >= 2 * c->n || !(h_galois[i] & 1))
        return fail(c, HE_EINVAL, "he_hma_plain: Galois element %d invalid", h_galois[i]);
    int32_t* g = ar.take<int32_t>(k);
    if (!g) return fail(c, HE_ENOMEM, "workspace too small");
    int e = upload(c, g, h_galois, (size_t)k * 4, S(stream));
    if (e) return e;
    d_gal = g;
  }
  dispatch_logn<LHmaPerm>(c->logn, c, acc, cts, k, pts, pt_stride, pt_limbs, d_gal, 1u, level, accumulate, 1,
                          S(stream));
  const int e = check_launch(c, "he_hma_plain");
  if (!e) *io_acc_scale = prod_scale;
  return e;
}

int he_hma_scalar(he_ctx* c, uint64_t* acc, const uint64_t* cts, int k, const int64_t* h_w, int level, int accumulate,
                  double ct_scale, double w_scale, double* io_acc_scale, void* stream) {
  if (!c || !acc || !cts || !h_w || !io_acc_scale || k < 1 || !level_ok(c, level))
    return fail(c, HE_EINVAL, "he_hma_scalar: bad arguments");
  const double prod_scale = ct_scale * w_scale;
  if (!scale_ok(ct_scale) || !scale_ok(w_scale) || !scale_ok(prod_scale) ||
      (accumulate && !scales_agree(*io_acc_scale, prod_scale)))
    return fail(c, HE_ESCALE, "he_hma_scalar: product scale %.17g does not match the accumulator's %.17g", prod_scale,
                *io_acc_scale);
  for (int i = 0; i < k; ++i)
    if (h_w[i] <= -(1ll << 62) || h_w[i] >= (1ll << 62)) return fail(c, HE_EINVAL, "he_hma_scalar: |w| >= 2^62");
  Arena ar(c);
  std::vector<int64_t> w(h_w, h_w + k);
  int e;
  if (!accumulate) {
    e = scalar_mac(c, acc, cts, k, w, 1, level, ar, S(stream));
  } else {
    u64* tmp = ar.take<u64>((size_t)2 * level * c->n);
    if (!tmp) return fail(c, HE_ENOMEM, "workspace too small");
    e = scalar_mac(c, tmp, cts, k, w, 1, level, ar, S(stream));
    if (!e) e = he_add(c, acc, acc, tmp, 1, level, prod_scale, prod_scale, stream);
  }
  if (!e) *io_acc_scale = prod_scale;
  return e;
}

int he_rescale(he_ctx* c, uint64_t* out, const uint64_t* in, int count, int level, void* stream) {
  if (!c || !out || !in || count < 1 || level < 2 || level > c->big_l || out == in)
    return fail(c, HE_EINVAL, "he_rescale: bad arguments");
  Arena ar(c);
  return rescale_batch(c, out, in, count, level, ar, S(stream));
}

int he_keygen_switch(he_ctx* c, int32_t galois, const uint64_t* d_s, const uint64_t* d_a, const int64_t* d_e,
                     uint64_t* d_key, void* stream) {
  if (!c || !d_s || !d_a || !d_e || !d_key) return fail(c, HE_EINVAL, "he_keygen_switch: null argument");
  if (c->capturing) return fail(c, HE_EUNSUPPORTED, "he_keygen_switch: not allowed during graph capture");
  if (galois != 0 && (galois < 1 || galois >= 2 * c->n || !(galois & 1)))
    return fail(c, HE_EINVAL, "he_keygen_switch: bad Galois element %d", galois);
  const int L = c->big_l;
  const size_t n = c->n;
  hipStream_t s = S(stream);
  // ehat[j][t] = NTT(e_j mod m_t)
  u64* ehat = nullptr;
  if (hipMalloc((void**)&ehat, (size_t)L * (L + 1) * n * 8) != hipSuccess) return fail(c, HE_ENOMEM, "keygen temp");
  for (int j = 0; j < L; ++j)
    k_from_signed<<<dim3(n / 256, L + 1), 256, 0, s>>>(ehat + (size_t)j * (L + 1) * n, d_e + (size_t)j * n, 0, (int)n,
                                                       c->mods);
  dispatch_logn<LNtt>(c->logn, c, ehat, L, L + 1, 0, true, s);
  ConstTable pm{};
  for (int t = 0; t < L; ++t) {
    pm.v[t] = c->moduli[L] % c->moduli[t];
    pm.sh[t] = shoup_companion(pm.v[t], c->moduli[t]);
  }
  dispatch_logn<LKeygen>(c->logn, c, (u64*)d_key, d_s, d_a, (const u64*)ehat, (u32)galois, pm, s, 0);
  int e = check_launch(c, "keygen");
  (void)hipStreamSynchronize(s);
  (void)hipFree(ehat);
  return e;
}

int he_keys_upload(he_ctx* c, const int32_t* h_galois, int n_keys, const uint64_t* keys, int keys_on_device,
                   void* stream) {
  if (!c || !h_galois || !keys || n_keys < 1) return fail(c, HE_EINVAL, "he_keys_upload: bad arguments");
  if (c->capturing) return fail(c, HE_EUNSUPPORTED, "he_keys_upload: not allowed during graph capture");
  for (int i = 0; i < n_keys; ++i) {
    const int32_t g = h_galois[i];
    if (g != 0 && (g < 1 || g >= 2 * c->n || !(g & 1) || g == 1))
      return fail(c, HE_EINVAL, "he_keys_upload: bad Galois element %d", g);
    for (int k = 0; k < i; ++k)
      if (h_galois[k] == g) return fail(c, HE_EINVAL, "he_keys_upload: Galois element %d listed twice", g);
  }
  const int L = c->big_l;
  const size_t key_elems = (size_t)L * 2 * (L + 1) * c->n;
  hipStream_t s = S(stream);
  std::vector<u64*> fresh(n_keys, nullptr);
  u64* staging = nullptr;
  int* bad = nullptr;
  auto cleanup = [&](bool drop_fresh) {
    (void)hipStreamSynchronize(s);
    if (drop_fresh)
      for (u64* k : fresh) (void)hipFree(k);
    (void)hipFree(staging);
    (void)hipFree(bad);
  };
  if (hipMalloc((void**)&bad, sizeof(int)) != hipSuccess ||
      (!keys_on_device && hipMalloc((void**)&staging, key_elems * 8) != hipSuccess)) {
    cleanup(true);
    return fail(c, HE_ENOMEM, "he_keys_upload: staging allocation failed");
  }
  (void)hipMemsetAsync(bad, 0, sizeof(int), s);
  for (int i = 0; i < n_keys; ++i) {
    if (hipMalloc((void**)&fresh[i], key_elems * 8) != hipSuccess) {
      fresh[i] = nullptr;
      cleanup(true);
      return fail(c, HE_ENOMEM, "he_keys_upload: key allocation failed");
    }
    const u64* src = keys + (size_t)i * key_elems;
    if (!keys_on_device) {
      // the staging buffer is reused by the next key only after this pack ran
      if (hipMemcpyAsync(staging, src, key_elems * 8, hipMemcpyHostToDevice, s) != hipSuccess) {
        cleanup(true);
        return fail(c, HE_EDEVICE, "he_keys_upload: host copy failed");
      }
      src = staging;
    }
    k_key_pack<<<dim3(c->n / 256, L + 1, 2 * L), 256, 0, s>>>(fresh[i], src, L, c->n, c->mods, bad);
    if (!keys_on_device) (void)hipStreamSynchronize(s);
  }
  int h_bad = 0;
  if (hipMemcpyAsync(&h_bad, bad, sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess || check_launch(c, "he_keys_upload") != HE_OK) {
    cleanup(true);
    return fail(c, HE_EDEVICE, "he_keys_upload: device failure");
  }
  if (h_bad) {
    cleanup(true);
    return fail(c, HE_EINVAL, "he_keys_upload: a key residue is not reduced modulo its prime");
  }
  bool replaced = false;
  for (int i = 0; i < n_keys; ++i) {
    auto it = c->keys.find(h_galois[i]);
    if (it != c->keys.end()) {
      replaced = true;
      (void)hipFree(it->second);
    }
    c->keys[h_galois[i]] = fresh[i];
  }
  if (replaced) ++c->epoch;
  cleanup(false);
  return HE_OK;
}

int he_has_key(const he_ctx* c, int32_t galois) { return c && c->keys.count(galois) ? 1 : 0; }

int he_keys_free(he_ctx* c, const int32_t* h_galois, int n_keys) {
  if (!c || n_keys < 0 || (n_keys > 0 && !h_galois)) return fail(c, HE_EINVAL, "he_keys_free: bad arguments");
  if (c->capturing) return fail(c, HE_EUNSUPPORTED, "he_keys_free: not allowed during graph capture");
  for (int i = 0; i < n_keys; ++i)
    if (!c->keys.count(h_galois[i])) return fail(c, HE_ENOKEY, "he_keys_free: no key for Galois element %d", h_galois[i]);
  ++c->epoch;
  (void)hipDeviceSynchronize();
  if (n_keys == 0) {
    for (auto& kv : c->keys) (void)hipFree(kv.second);
    c->keys.clear();
    return HE_OK;
  }
  for (int i = 0; i < n_keys; ++i) {
    auto it = c->keys.find(h_galois[i]);
    (void)hipFree(it->second);
    c->keys.erase(it);
  }
  return HE_OK;
}

int he_from_signed(he_ctx* c, uint64_t* d_out, const int64_t* d_coeffs, int n_limbs, int first_mod, void* stream) {
  if (!c || !d_out || !d_coeffs || n_limbs < 1 || first_mod < 0 || first_mod + n_limbs > c->big_l + 1)
    return fail(c, HE_EINVAL, "he_from_signed: bad arguments");
  k_from_signed<<<dim3(c->n / 256, n_limbs), 256, 0, S(stream)>>>(d_out, d_coeffs, first_mod, c->n, c->mods);
  return check_launch(c, "he_from_signed");
}

int he_encrypt_sk(he_ctx* c, uint64_t* d_ct, const uint64_t* d_pt, const uint64_t* d_a, const int64_t* d_e,
                  const uint64_t* d_s, int level, void* stream) {
  if (!c || !d_ct || !d_pt || !d_a || !d_e || !d_s || !level_ok(c, level))
    return fail(c, HE_EINVAL, "he_encrypt_sk: bad arguments");
  Arena ar(c);
  u64* ehat = ar.take<u64>((size_t)level * c->n);
  if (!ehat) return fail(c, HE_ENOMEM, "workspace too small");
  hipStream_t s = S(stream);
  k_from_signed<<<dim3(c->n / 256, level), 256, 0, s>>>(ehat, d_e, 0, c->n, c->mods);
  dispatch_logn<LNtt>(c->logn, c, ehat, 1, level, 0, true, s);
  k_encrypt<<<dim3(c->n / 256, level), 256, 0, s>>>(d_ct, d_pt, d_a, ehat, d_s, level, c->n, c->mods);
  return check_launch(c, "he_encrypt_sk");
}

int he_decrypt(he_ctx* c, uint64_t* d_out, const uint64_t* d_ct, const uint64_t* d_s, int level, void* stream) {
  if (!c || !d_out || !d_ct || !d_s || !level_ok(c, level)) return fail(c, HE_EINVAL, "he_decrypt: bad arguments");
  k_decrypt<<<dim3(c->n / 256, level), 256, 0, S(stream)>>>(d_out, d_ct, d_s, level, c->n, c->mods);
  return check_launch(c, "he_decrypt");
}

int he_encode_coeffs(int n, const double* h_z, int n_values, double scale, int64_t* h_out) {
  if (!h_z || !h_out) return HE_EINVAL;
  return encode_coeffs(n, h_z, n_values, scale, h_out) ? HE_EINVAL : HE_OK;
}

int he_decode_coeffs(int n, const double* h_m, int n_values, double* h_z) {
  if (!h_m || !h_z) return HE_EINVAL;
  return decode_coeffs(n, h_m, n_values, h_z) ? HE_EINVAL : HE_OK;
}

int he_rotate(he_ctx* c, uint64_t* d_out, const uint64_t* d_in, int count, int level, int k, void* stream) {
  if (!c || !d_out || !d_in || count < 1 || !level_ok(c, level)) return fail(c, HE_EINVAL, "he_rotate: bad arguments");
  Arena ar(c);
  return rotate_batch(c, d_out, d_in, count, level, k, EPI_ROT, ar, S(stream));
}

int he_rotate_static(he_ctx* c, uint64_t* d_out, const uint64_t* d_in, int count, int level, int k, void* stream) {
  if (!c || !d_out || !d_in || count < 1 || !level_ok(c, level))
    return fail(c, HE_EINVAL, "he_rotate_static: bad arguments");
  if (!c->fixed_scratch) return fail(c, HE_EDEVICE, "he_rotate_static: no scratch array on this device");
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != c->device)
    return fail(c, HE_EINVAL, "he_rotate_static: the context's device (%d) is not current (%d)", c->device, dev);
  // one ciphertext's key-switch temporaries must fit; larger batches run in chunks
  const size_t one = (ks_elems_per_job(level, p_groups(c, level), c->n) + 128) * 8;
  if (one > STATIC_SCRATCH_BYTES)
    return fail(c, HE_ENOMEM, "he_rotate_static: one ciphertext at level %d needs %zu bytes of scratch (max %zu)",
                level, one, STATIC_SCRATCH_BYTES);
  Arena ar(c->fixed_scratch, STATIC_SCRATCH_BYTES);
  return rotate_batch(c, d_out, d_in, count, level, k, EPI_ROT, ar, S(stream));
}

int he_rotate_static_max_batch(const he_ctx* c, int level) {
  if (!c || !level_ok(const_cast<he_ctx*>(c), level)) return HE_EINVAL;
  Arena ar(c->fixed_scratch, STATIC_SCRATCH_BYTES);
  return chunk_for(ar, 1 << 30, level, p_groups(c, level), c->n);
}

int he_rotsum(he_ctx* c, uint64_t* d_cts, int count, int level, int r_steps, void* stream) {
  if (!c || !d_cts || count < 1 || r_steps < 0 || r_steps > 20 || !level_ok(c, level))
    return fail(c, HE_EINVAL, "he_rotsum: bad arguments");
  Arena ar(c);
  for (int j = 0; j < r_steps; ++j) {
    int e = rotate_batch(c, d_cts, d_cts, count, level, 1 << j, EPI_ROTSUM, ar, S(stream));
    if (e) return e;
  }
  return HE_OK;
}

int he_batch_rotate(he_ctx* c, uint64_t* const* h_outs, const uint64_t* const* h_ins, const int32_t* h_levels,
                    const int32_t* h_steps, int count, int accumulate, void* stream) {
  if (!c || !h_outs || !h_ins || !h_levels || !h_steps || count < 1)
    return fail(c, HE_EINVAL, "he_batch_rotate: null argument");
  std::vector<KsJob> jobs(count);
  for (int b = 0; b < count; ++b) {
    const int level = h_levels[b];
    if (!level_ok(c, level) || !h_outs[b] || !h_ins[b]) return fail(c, HE_EINVAL, "he_batch_rotate: bad item %d", b);
    const u32 g = galois_of(h_steps[b], c->n);
    const u64* key = nullptr;
    if (g != 1) {
      auto it = c->keys.find((int)g);
      if (it == c->keys.end()) return fail(c, HE_ENOKEY, "he_batch_rotate: no key for step %d", h_steps[b]);
      key = it->second;
    }
    jobs[b] = KsJob{h_ins[b] + (size_t)level * c->n, h_ins[b], h_outs[b], key, g, galois_of(-h_steps[b], c->n),
                    level, 0};
  }
  Arena ar(c);
  return rotate_jobs(c, jobs, accumulate ? EPI_ROTSUM : EPI_ROT, ar, S(stream));
}

int he_batch_rescale(he_ctx* c, uint64_t* const* h_outs, const uint64_t* const* h_ins, const int32_t* h_levels,
                     int count, void* stream) {
  if (!c || !h_outs || !h_ins || !h_levels || count < 1) return fail(c, HE_EINVAL, "he_batch_rescale: null argument");
  std::vector<KsJob> jobs(count);
  int lmax = 2;
  for (int b = 0; b < count; ++b) {
    const int level = h_levels[b];
    if (level < 2 || level > c->big_l || !h_outs[b] || !h_ins[b] || h_outs[b] == h_ins[b])
      return fail(c, HE_EINVAL, "he_batch_rescale: bad item %d", b);
    jobs[b] = KsJob{h_ins[b], h_ins[b], h_outs[b], nullptr, 1u, 1u, level, 0};
    lmax = std::max(lmax, level);
  }
  const int n = c->n;
  hipStream_t s = S(stream);
  Arena ar(c);
  const int chunk = (int)std::min<size_t>({(size_t)count, ar.left() / 8 / (2 * (size_t)n + 64), (size_t)32000});
  if (chunk < 1) return fail(c, HE_ENOMEM, "workspace too small for rescale");
  KsJob* d_jobs = ar.take<KsJob>(chunk);
  u64* rc = ar.take<u64>((size_t)chunk * 2 * n);
  if (!d_jobs || !rc) return fail(c, HE_ENOMEM, "workspace too small for rescale");
  for (int b0 = 0; b0 < count; b0 += chunk) {
    const int cn = std::min(chunk, count - b0);
    int e = upload(c, d_jobs, jobs.data() + b0, (size_t)cn * sizeof(KsJob), s);
    if (e) return e;
    dispatch_logn<LIntt1>(c->logn, c, (const KsJob*)d_jobs, cn, lmax, rc, s);
    dispatch_logn<LDrop>(c->logn, c, (int)MODE_LAST, (int)EPI_STORE, (const KsJob*)d_jobs, cn, lmax, 0,
                         (const u64*)nullptr, (const u64*)rc, s);
  }
  return check_launch(c, "he_batch_rescale");
}

int he_batch_mul_plain(he_ctx* c, uint64_t* const* h_outs, const uint64_t* const* h_cts, const uint64_t* const* h_pts,
                       const int32_t* h_levels, int count, void* stream) {
  if (!c || !h_outs || !h_cts || !h_pts || !h_levels || count < 1 || count > 65535)
    return fail(c, HE_EINVAL, "he_batch_mul_plain: bad arguments");
  std::vector<KsJob> jobs(count);
  int lmax = 1;
  for (int b = 0; b < count; ++b) {
    if (!level_ok(c, h_levels[b]) || !h_outs[b] || !h_cts[b] || !h_pts[b])
      return fail(c, HE_EINVAL, "he_batch_mul_plain: bad item %d", b);
    jobs[b] = KsJob{h_cts[b], h_pts[b], h_outs[b], nullptr, 1u, 1u, h_levels[b], 0};
    lmax = std::max(lmax, h_levels[b]);
  }
  hipStream_t s = S(stream);
  Arena ar(c);
  KsJob* d_jobs = ar.take<KsJob>(count);
  if (!d_jobs) return fail(c, HE_ENOMEM, "workspace too small");
  int e = upload(c, d_jobs, jobs.data(), (size_t)count * sizeof(KsJob), s);
  if (e) return e;
  Prof pr(c, "batch_mul_plain", s);
  k_batch_mul_plain<<<dim3(c->n / 256, lmax, count), 256, 0, s>>>(d_jobs, c->n, c->mods);
  return check_launch(c, "he_batch_mul_plain");
}

int he_combine_cp_dp_batch(he_ctx* c, int count, const uint64_t* d_in, int o_c, int level, int spatial,
                           int per_dense, uint64_t* d_out, void* stream) {
  if (!c || !d_in || !d_out || count < 1 || o_c < 1 || spatial < 1 || per_dense < 1 || !level_ok(c, level) ||
      (long long)per_dense * spatial > c->n / 2)
    return fail(c, HE_EINVAL, "he_combine_cp_dp: bad arguments");
  const int n = c->n;
  const int n_dense = (o_c + per_dense - 1) / per_dense;
  if ((long long)count * n_dense > 65535) return fail(c, HE_EINVAL, "he_combine_cp_dp: too many items");
  const size_t cstride = (size_t)2 * level * n;
  hipStream_t s = S(stream);
  Arena ar(c);
  const size_t total = (size_t)count * o_c;
  u64* rot = ar.take<u64>(total * cstride);
  if (!rot) return fail(c, HE_ENOMEM, "workspace too small for combine");
  std::vector<KsJob> jobs(total);
  int64_t n_rot = 0;
  for (int o = 0; o < o_c; ++o) {
    const int step = -(o % per_dense) * spatial;
    const u32 g = galois_of(step, n);
    const u64* key = nullptr;
    if (g != 1) {
      auto it = c->keys.find((int)g);
      if (it == c->keys.end()) return fail(c, HE_ENOKEY, "he_combine_cp_dp: no key for step %d", step);
      key = it->second;
      n_rot += count;
    }
    for (int b = 0; b < count; ++b) {
      const size_t idx = (size_t)b * o_c + o;
      const u64* in = d_in + idx * cstride;
      jobs[idx] = KsJob{in + (size_t)level * n, in, rot + idx * cstride, key, g, galois_of(-step, n), level, 0};
    }
  }
  int e = rotate_jobs(c, jobs, EPI_ROT, ar, s);
  if (e) return e;
  {
    Prof pr(c, "block_sum", s);
    k_block_sum<<<dim3(n / 256, level, count * n_dense), 256, 0, s>>>(d_out, rot, o_c, per_dense, n_dense, level, n,
                                                                      c->mods);
  }
  c->counts = he_counts{};
  c->counts.rot = n_rot;
  c->counts.addcc = (int64_t)count * (o_c - n_dense);
  return check_launch(c, "he_combine_cp_dp");
}

int he_combine_cp_dp(he_ctx* c, const uint64_t* d_in, int o_c, int level, int spatial, int per_dense,
                     uint64_t* d_out, void* stream) {
  return he_combine_cp_dp_batch(c, 1, d_in, o_c, level, spatial, per_dense, d_out, stream);
}

int he_gather_onehot(he_ctx* c, int count, const uint64_t* d_cts, int k, const uint64_t* d_mask, int level,
                     uint64_t* d_out, void* stream) {
  if (!c || !d_cts || !d_mask || !d_out || count < 1 || count > 65535 || k < 1 || k > c->n / 2 || !level_ok(c, level))
    return fail(c, HE_EINVAL, "he_gather_onehot: bad arguments");
  const u32 g5inv = galois_of(-1, c->n);
  dispatch_logn<LHmaPerm>(c->logn, c, d_out, d_cts, k, d_mask, 0, level, (const int32_t*)nullptr, g5inv, level, 0,
                          count, S(stream));
  c->counts = he_counts{};
  c->counts.mulpc = (int64_t)count * k;
  c->counts.addcc = (int64_t)count * (k - 1);
  return check_launch(c, "he_gather_onehot");
}

int he_rotate_hoisted(he_ctx* c, const uint64_t* d_in, int level, const int32_t* h_steps, int m, uint64_t* d_outs,
                      void* stream) {
  if (!c || !d_in || !h_steps || !d_outs || m < 1 || m > 32000 || !level_ok(c, level))
    return fail(c, HE_EINVAL, "he_rotate_hoisted: bad arguments");
  const int n = c->n;
  std::vector<KsJob> jobs(m);
  for (int r = 0; r < m; ++r) {
    const u32 g = galois_of(h_steps[r], n);
    auto it = c->keys.find((int)g);
    if (g == 1 || it == c->keys.end())
      return fail(c, g == 1 ? HE_EINVAL : HE_ENOKEY, "he_rotate_hoisted: no key for step %d", h_steps[r]);
    jobs[r] = KsJob{d_in + (size_t)level * n, d_in, d_outs + (size_t)r * 2 * level * n, it->second, g,
                    galois_of(-h_steps[r], n), level, 0};
  }
  hipStream_t s = S(stream);
  Arena ar(c);
  KsJob* job1 = ar.take<KsJob>(1);
  u64* dcoef = ar.take<u64>((size_t)level * n);
  u64* dhat = ar.take<u64>((size_t)level * (level + 1) * n);
  KsJob* d_jobs = ar.take<KsJob>(m);
  // fused: per rotation only the coefficient-domain P limb (2 N); else also
  // the 2 (level + 1) inner-product rows
  const bool fused = c->hoist_fused != 0;
  const size_t per = (fused ? 0 : (size_t)2 * (level + 1) * n) + 2 * (size_t)n;
  const int chunk = (int)std::min<size_t>((size_t)m, ar.left() / 8 / (per + 64));
  if (!job1 || !dcoef || !dhat || !d_jobs || chunk < 1)
    return fail(c, HE_ENOMEM, "workspace too small for hoisted rotation");
  u64* u = fused ? nullptr : ar.take<u64>((size_t)chunk * 2 * (level + 1) * n);
  u64* rc = ar.take<u64>((size_t)chunk * 2 * n);
  // the digits of c1 itself: a job with no permutation
  KsJob j1 = jobs[0];
  j1.g = j1.ginv = 1;
  int e = upload(c, job1, &j1, sizeof(KsJob), s);
  if (!e) e = upload(c, d_jobs, jobs.data(), (size_t)m * sizeof(KsJob), s);
  if (e) return e;
  dispatch_logn<LHoistUp>(c->logn, c, (const KsJob*)job1, 1, level, dcoef, dhat, s);
  if (!fused && chunk == m) {
    hoisted_rest(c, d_jobs, m, level, dhat, u, rc, s, 1 << 30, 0);
    return check_launch(c, "he_rotate_hoisted");
  }
  for (int r0 = 0; r0 < m; r0 += chunk) {
    const int cm = std::min(chunk, m - r0);
    dispatch_logn<LHoisted>(c->logn, c, (const KsJob*)(d_jobs + r0), cm, level, (const u64*)dhat, u, rc, s);
  }
  return check_launch(c, "he_rotate_hoisted");
}

int he_rotate_hoisted_batch(he_ctx* c, const uint64_t* d_in, int count, int level, const int32_t* h_steps, int m,
                            uint64_t* d_outs, void* stream) {
  if (!c || !d_in || !h_steps || !d_outs || count < 1 || m < 1 || m > MAX_HOIST || !level_ok(c, level))
    return fail(c, HE_EINVAL, "he_rotate_hoisted_batch: bad arguments");
  if ((long long)count * m > ((long long)1 << 31) / (2 * level * (long long)c->n))
    return fail(c, HE_EINVAL, "he_rotate_hoisted_batch: too many outputs");
  const int n = c->n;
  HoistKeys hk{};
  for (int r = 0; r < m; ++r) {
    const u32 g = galois_of(h_steps[r], n);
    auto it = c->keys.find((int)g);
    if (g == 1 || it == c->keys.end())
      return fail(c, g == 1 ? HE_EINVAL : HE_ENOKEY, "he_rotate_hoisted_batch: no key for step %d", h_steps[r]);
    hk.key[r] = it->second;
    hk.g[r] = g;
    hk.ginv[r] = galois_of(-h_steps[r], n);
  }
  Arena ar(c);
  return hoisted_batch(c, d_in, (size_t)2 * level * n, count, level, hk, m, d_outs, ar, S(stream));
}

size_t he_tap_workspace_need(he_ctx* c, int n_batch, int level, const he_conv_desc* desc, int o_c2, int square) {
  if (!c || !desc || n_batch < 1 || level < 2 || level > c->big_l) return 0;
  TapPlan tp;
  if (tap_plan(c, "he_tap_workspace_need", desc, tp, false)) return 0;
  size_t need = tap_need(c, tp, n_batch, level);
  if (o_c2 > 0) {  // the FFConv tail after the r W1 outputs at level - 1
    auto al = [](size_t elems) { return ((elems * 8 + 255) & ~(size_t)255); };
    const size_t n = c->n, l1 = level - 1, l2 = level - 2, nb = n_batch;
    need += al(nb * desc->o_c * 2 * l1 * n) * 2 + al(nb * o_c2 * 2 * l1 * n) +
            (square ? 2 * al(nb * o_c2 * 2 * l2 * n) : 0) + al(2 * (size_t)desc->o_c * o_c2 * l1);
  }
  return need;
}

int he_conv_tap(he_ctx* c, int n_batch, const uint64_t* d_in, int level, const he_conv_desc* desc,
                const uint64_t* d_filt, int pt_limbs, const uint64_t* d_filt_p, double in_scale, double pt_scale,
                uint64_t* d_out, double* out_scale, void* stream) {
  if (!c || !d_in || !desc || !d_filt || !d_out || !out_scale || n_batch < 1 || pt_limbs < 1)
    return fail(c, HE_EINVAL, "he_conv_tap: bad arguments");
  if (level < 2 || level > c->big_l) return fail(c, HE_ELEVEL, "he_conv_tap needs 2 <= level <= L (got %d)", level);
  if (pt_limbs < level) return fail(c, HE_EINVAL, "he_conv_tap: plaintexts have %d limbs, level is %d", pt_limbs, level);
  if (!scale_ok(in_scale) || !scale_ok(pt_scale))
    return fail(c, HE_ESCALE, "he_conv_tap: scales %.17g, %.17g", in_scale, pt_scale);
  TapPlan tp;
  int e = tap_plan(c, "he_conv_tap", desc, tp);
  if (e) return e;
  if ((long long)n_batch * desc->o_c > 65535 || (long long)n_batch * tp.m_cts > 65535)
    return fail(c, HE_EINVAL, "he_conv_tap: batch too large for one call");
  c->counts = he_counts{};
  Arena ar(c);
  e = tap_run(c, tp, n_batch, d_in, level, d_filt, pt_limbs, d_filt_p, d_out, ar, S(stream));
  if (!e) *out_scale = in_scale * pt_scale / (double)c->moduli[level - 1];
  return e;
}

int ffconv_layer_tap(he_ctx* c, int n_batch, const uint64_t* d_in, int level, const he_conv_desc* desc,
                     const uint64_t* d_w1, int w1_limbs, const uint64_t* d_w1_p, double in_scale, double w1_scale,
                     const uint64_t* d_mask,
                     double mask_scale, const double* h_w2, const uint64_t* d_w2_tab, int o_c2, int k_bits,
                     int square, uint64_t* d_out, double* out_scale, void* stream) {
  if (!c || !d_in || !desc || !d_w1 || !d_mask || (!h_w2 && !d_w2_tab) || !d_out || !out_scale || n_batch < 1 ||
      o_c2 < 1 || k_bits < 0 || k_bits > 40 || w1_limbs < 1)
    return fail(c, HE_EINVAL, "ffconv_layer_tap: bad arguments");
  const int need = square ? 4 : 3;
  if (level < need || level > c->big_l)
    return fail(c, HE_ELEVEL, "ffconv_layer_tap needs %d <= level <= L (got %d)", need, level);
  if (w1_limbs < level) return fail(c, HE_EINVAL, "ffconv_layer_tap: W1 plaintexts have %d limbs, level is %d", w1_limbs, level);
  if (square && !c->keys.count(0)) return fail(c, HE_ENOKEY, "ffconv_layer_tap: no relinearisation key");
  if (!scale_ok(in_scale) || !scale_ok(w1_scale) || !scale_ok(mask_scale))
    return fail(c, HE_ESCALE, "ffconv_layer_tap: scales %.17g, %.17g, %.17g", in_scale, w1_scale, mask_scale);
  TapPlan tp;
  int e = tap_plan(c, "ffconv_layer_tap", desc, tp);
  if (e) return e;
  const int r = desc->o_c;
  if ((long long)n_batch * r > 65535 || (long long)n_batch * o_c2 > 65535 || (long long)n_batch * tp.m_cts > 65535)
    return fail(c, HE_EINVAL, "ffconv_layer_tap: batch too large for one call");
  const int n = c->n;
  hipStream_t s = S(stream);
  c->counts = he_counts{};
  Arena ar(c);
  const u64* d_tab = d_w2_tab;
  if (!d_w2_tab) {  // from host weights: one copy to the device, so not capturable
    std::vector<int64_t> w((size_t)r * o_c2);
    for (size_t i = 0; i < w.size(); ++i) {
      const double x = std::ldexp(h_w2[i], k_bits);
      if (!(std::fabs(x) < 4.0e18)) return fail(c, HE_EINVAL, "ffconv_layer_tap: W2 weight not finite or too large");
      w[i] = round_half_away(x);
    }
    std::vector<u64> tab = scalar_table(c, w, level - 1);
    u64* t = ar.take<u64>(tab.size());
    if (!t) return fail(c, HE_ENOMEM, "workspace too small for ffconv_layer_tap");
    if ((e = upload(c, t, tab.data(), tab.size() * 8, s))) return e;
    d_tab = t;
  }
  u64* y = ar.take<u64>((size_t)n_batch * r * 2 * (level - 1) * n);
  if (!y) return fail(c, HE_ENOMEM, "workspace too small for ffconv_layer_tap");
  if ((e = tap_run(c, tp, n_batch, d_in, level, d_w1, w1_limbs, d_w1_p, y, ar, s))) return e;
  if ((e = ffconv_tail(c, n_batch, y, level - 1, 1, r, d_mask, d_tab, o_c2, square, d_out, ar, s, true))) return e;
  const double y_scale = in_scale * w1_scale / (double)c->moduli[level - 1];
  double z_scale = y_scale * mask_scale * std::ldexp(1.0, k_bits) / (double)c->moduli[level - 2];
  if (square) z_scale = z_scale * z_scale / (double)c->moduli[level - 3];
  *out_scale = z_scale;
  return HE_OK;
}

size_t he_him2col_workspace_need(he_ctx* c, int n_batch, int level, const he_conv_desc* desc) {
  if (!c || !desc || n_batch < 1 || level < 2 || level > c->big_l) return 0;
  Him2colPlan hp;
  if (him2col_plan(c, desc, hp, false)) return 0;
  return him2col_need(c, hp, n_batch, level);
}

int he_him2col(he_ctx* c, int n_batch, const uint64_t* d_in, int level, const he_conv_desc* desc,
               const uint64_t* d_masks, int mask_limbs, double in_scale, double mask_scale, uint64_t* d_out,
               double* out_scale, void* stream) {
  if (!c || !d_in || !desc || !d_masks || !d_out || !out_scale || n_batch < 1 || mask_limbs < 1)
    return fail(c, HE_EINVAL, "he_him2col: bad arguments");
  if (level < 2 || level > c->big_l) return fail(c, HE_ELEVEL, "he_him2col needs 2 <= level <= L (got %d)", level);
  if (mask_limbs < level) return fail(c, HE_EINVAL, "he_him2col: masks have %d limbs, level is %d", mask_limbs, level);
  if (!scale_ok(in_scale) || !scale_ok(mask_scale))
    return fail(c, HE_ESCALE, "he_him2col: scales %.17g, %.17g", in_scale, mask_scale);
  Him2colPlan hp;
  int e = him2col_plan(c, desc, hp);
  if (e) return e;
  const int kk = hp.map.d2 * desc->c_in;
  if ((long long)n_batch * kk > 65535) return fail(c, HE_EINVAL, "he_him2col: more than 65535 outputs in one call");
  const int n = c->n;
  const size_t cs = (size_t)2 * level * n;
  hipStream_t s = S(stream);
  c->counts = he_counts{};
  Arena ar(c);
  u64* z = ar.take<u64>((size_t)n_batch * hp.m_cts * hp.per * cs);
  u64* rot = hp.nrot ? ar.take<u64>((size_t)n_batch * hp.map.nvalid * hp.nrot * cs) : nullptr;
  u64* tmp = ar.take<u64>((size_t)n_batch * kk * cs);
  if (!z || (hp.nrot && !rot) || !tmp) return fail(c, HE_ENOMEM, "workspace too small for he_him2col");
  for (int b = 0; b < n_batch; ++b) {
    const u64* xb = d_in + (size_t)b * hp.m_cts * cs;
    u64* zb = z + (size_t)b * hp.m_cts * hp.per * cs;
    // z[b][m][0] = x_m; z[b][m][blk] = Rot(x_m, blk H W), hoisted per x_m
    if (hipMemcpy2DAsync(zb, hp.per * cs * 8, xb, cs * 8, cs * 8, hp.m_cts, hipMemcpyDeviceToDevice, s) != hipSuccess)
      return fail(c, HE_EDEVICE, "he_him2col: device copy failed");
    if (hp.m_cts > 1 && hp.nblk > 0 &&
        (e = hoisted_batch(c, xb, cs, hp.m_cts - 1, level, hp.blk, hp.nblk, zb + cs, ar, s, hp.per * cs)))
      return e;
    if (hp.last > 1 && (e = hoisted_batch(c, xb + (size_t)(hp.m_cts - 1) * cs, cs, 1, level, hp.blk, hp.last - 1,
                                          zb + ((size_t)(hp.m_cts - 1) * hp.per + 1) * cs, ar, s, hp.per * cs)))
      return e;
    // every valid block-shifted ciphertext rotated by the nonzero tap shifts, hoisted per ciphertext
    if (hp.nrot && (e = hoisted_batch(c, zb, cs, hp.map.nvalid, level, hp.tap, hp.nrot,
                                      rot + (size_t)b * hp.map.nvalid * hp.nrot * cs, ar, s)))
      return e;
  }
  k_him2col_mask<<<dim3(n / 256, level, n_batch * kk), 256, 0, s>>>(z, rot, d_masks, mask_limbs, tmp, level, n,
                                                                     hp.map, c->mods);
  if ((e = check_launch(c, "he_him2col masks"))) return e;
  if ((e = rescale_batch(c, d_out, tmp, n_batch * kk, level, ar, s))) return e;
  c->counts.rot += (int64_t)n_batch * ((int64_t)(hp.m_cts - 1) * hp.nblk + (hp.last - 1) +
                                       (int64_t)hp.map.nvalid * hp.nrot);
  c->counts.mulpc += (int64_t)n_batch * kk;
  c->counts.rescale += (int64_t)n_batch * kk;
  *out_scale = in_scale * mask_scale / (double)c->moduli[level - 1];
  return HE_OK;
}

int he_square(he_ctx* c, uint64_t* d_out, const uint64_t* d_in, int count, int level, void* stream) {
  if (!c || !d_out || !d_in || count < 1 || !level_ok(c, level)) return fail(c, HE_EINVAL, "he_square: bad arguments");
  Arena ar(c);
  return square_batch(c, d_out, d_in, count, level, ar, S(stream));
}

int he_conv_densepack(he_ctx* c, const uint64_t* d_in, int level, const he_conv_desc* desc, const uint64_t* d_filt,
                      uint64_t* d_out, void* stream) {
  if (!c || !d_in || !desc || !d_filt || !d_out) return fail(c, HE_EINVAL, "he_conv_densepack: null argument");
  c->counts = he_counts{};
  Arena ar(c);
  return densepack_run(c, d_in, level, desc, d_filt, d_out, ar, S(stream));
}

int he_conv_densepack_batch(he_ctx* c, int n_layers, const uint64_t* d_in, size_t in_stride, int level,
                            const he_conv_desc* desc, const uint64_t* d_filt, size_t filt_stride, uint64_t* d_out,
                            void* stream) {
  if (!c || !d_in || !desc || !d_filt || !d_out || n_layers < 1)
    return fail(c, HE_EINVAL, "he_conv_densepack_batch: bad arguments");
  c->counts = he_counts{};
  Arena ar(c);
  return densepack_run(c, d_in, level, desc, d_filt, d_out, ar, S(stream), n_layers, in_stride, filt_stride);
}

// Integer weights of a ConvPack layer whose rescale by q_{level-1} lands on
// target: round-half-away(w * (q_{level-1} target / in_scale)).  Checks the
// scales and the weights' range before anything is launched.
int convpack_weights(he_ctx* c, const char* who, const double* h_w, size_t count, int level, double in_scale,
                     double target_scale, std::vector<int64_t>& w, double& w_scale) {
  const double q_last = (double)c->moduli[level - 1];
  w_scale = q_last * target_scale / in_scale;
  if (!scale_ok(in_scale) || !scale_ok(target_scale) || !std::isfinite(w_scale) || w_scale < 1.0)
    return fail(c, HE_ESCALE, "%s: input scale %.17g cannot reach target %.17g at level %d", who, in_scale,
                target_scale, level);
  w.resize(count);
  for (size_t i = 0; i < count; ++i) {
    const double x = h_w[i] * w_scale;
    if (!(std::fabs(x) < 4.0e18)) return fail(c, HE_EINVAL, "%s: weight too large for the scale", who);
    w[i] = round_half_away(x);
  }
  return HE_OK;
}

// One ConvPack layer (Table II): out[o] = rescale(sum_k w[k][o] in[k]); adds
// its counts.  z: o_c ciphertexts of workspace at `level`.
int convpack_run(he_ctx* c, const u64* in, int k, int level, const std::vector<int64_t>& w, int o_c, u64* out,
                 Arena& ar, hipStream_t s) {
  u64* z = ar.take<u64>((size_t)o_c * 2 * level * c->n);
  if (!z) return fail(c, HE_ENOMEM, "workspace too small for ConvPack");
  int e = scalar_mac(c, z, in, k, w, o_c, level, ar, s);
  if (!e) e = rescale_batch(c, out, z, o_c, level, ar, s);
  c->counts.mulpc += (int64_t)k * o_c;
  c->counts.addcc += (int64_t)(k - 1) * o_c;
  c->counts.rescale += o_c;
  return e;
}

int he_conv_convpack(he_ctx* c, const uint64_t* d_in, int k, int level, const double* h_w, int o_c, double in_scale,
                     double target_scale, uint64_t* d_out, double* out_scale, void* stream) {
  if (!c || !d_in || !h_w || !d_out || !out_scale || k < 1 || o_c < 1 || o_c > 65535)
    return fail(c, HE_EINVAL, "he_conv_convpack: bad arguments");
  if (level < 2 || level > c->big_l) return fail(c, HE_ELEVEL, "he_conv_convpack needs 2 <= level <= L (got %d)", level);
  std::vector<int64_t> w;
  double w_scale = 0;
  int e = convpack_weights(c, "he_conv_convpack", h_w, (size_t)k * o_c, level, in_scale, target_scale, w, w_scale);
  if (e) return e;
  c->counts = he_counts{};
  Arena ar(c);
  e = convpack_run(c, d_in, k, level, w, o_c, d_out, ar, S(stream));
  if (!e) *out_scale = in_scale * w_scale / (double)c->moduli[level - 1];
  return e;
}

int ffconv_layer_convpack(he_ctx* c, const uint64_t* d_in, int k, int level, const double* h_w1, int r,
                          const double* h_w2, int o_c, double in_scale, double target_scale, int square,
                          uint64_t* d_out, double* out_scale, void* stream) {
  if (!c || !d_in || !h_w1 || !h_w2 || !d_out || !out_scale || k < 1 || r < 1 || o_c < 1 || r > 65535 ||
      o_c > 65535)
    return fail(c, HE_EINVAL, "ffconv_layer_convpack: bad arguments");
  const int need = square ? 4 : 3;
  if (level < need || level > c->big_l)
    return fail(c, HE_ELEVEL, "ffconv_layer_convpack needs %d <= level <= L (got %d)", need, level);
  if (square && !c->keys.count(0)) return fail(c, HE_ENOKEY, "ffconv_layer_convpack: no relinearisation key");
  // W1 lands on target_scale; W2 on target_scale, or with x^2 on the scale
  // whose square, rescaled by q_{level-3}, is target_scale
  const double t2 = square ? std::sqrt((double)c->moduli[level - 3] * target_scale) : target_scale;
  std::vector<int64_t> w1, w2;
  double s1 = 0, s2 = 0;
  int e = convpack_weights(c, "ffconv_layer_convpack (W1)", h_w1, (size_t)k * r, level, in_scale, target_scale, w1, s1);
  if (e) return e;
  const double y_scale = in_scale * s1 / (double)c->moduli[level - 1];
  e = convpack_weights(c, "ffconv_layer_convpack (W2)", h_w2, (size_t)r * o_c, level - 1, y_scale, t2, w2, s2);
  if (e) return e;
  double z_scale = y_scale * s2 / (double)c->moduli[level - 2];
  const int n = c->n;
  c->counts = he_counts{};
  Arena ar(c);
  hipStream_t s = S(stream);
  u64* y = ar.take<u64>((size_t)r * 2 * (level - 1) * n);
  u64* z = square ? ar.take<u64>((size_t)o_c * 2 * (level - 2) * n) : d_out;
  u64* sq = square ? ar.take<u64>((size_t)o_c * 2 * (level - 2) * n) : nullptr;
  if (!y || !z || (square && !sq)) return fail(c, HE_ENOMEM, "workspace too small for ffconv_layer_convpack");
  // W1 under ConvPack; its r channel ciphertexts are W2's ConvPack inputs as
  // they stand (HGrouping with d = 1: no slot moves, no rotation)
  e = convpack_run(c, d_in, k, level, w1, r, y, ar, s);
  if (!e) e = convpack_run(c, y, r, level - 1, w2, o_c, z, ar, s);
  if (!e && square) {
    e = square_batch(c, sq, z, o_c, level - 2, ar, s);
    if (!e) e = rescale_batch(c, d_out, sq, o_c, level - 2, ar, s);
    c->counts.square += o_c;
    c->counts.rescale += o_c;
    z_scale = z_scale * z_scale / (double)c->moduli[level - 3];
  }
  if (!e) *out_scale = z_scale;
  return e;
}

int ffconv_layer(he_ctx* c, const uint64_t* d_in, int level, const he_conv_desc* desc, const uint64_t* d_w1_filt,
                 const uint64_t* d_mask, const double* h_w2, int o_c2, int k_bits, int square, uint64_t* d_out,
                 void* stream) {
  if (!c || !d_in || !desc || !d_w1_filt || !d_mask || !h_w2 || !d_out)
    return fail(c, HE_EINVAL, "ffconv_layer: null argument");
  if (o_c2 < 1 || k_bits < 0 || k_bits > 40 || desc->o_c < 1) return fail(c, HE_EINVAL, "ffconv_layer: bad W2 shape or k_bits");
  if (level < 3 || level > c->big_l) return fail(c, HE_ELEVEL, "ffconv_layer needs level >= 3 (got %d)", level);
  std::vector<int64_t> w((size_t)desc->o_c * o_c2);
  for (size_t i = 0; i < w.size(); ++i) {
    const double x = std::ldexp(h_w2[i], k_bits);
    if (!(std::fabs(x) < 4.0e18)) return fail(c, HE_EINVAL, "ffconv_layer: W2 weight not finite or too large");
    w[i] = round_half_away(x);
  }
  std::vector<u64> tab = scalar_table(c, w, level - 1);
  Arena ar(c);
  u64* d_tab = ar.take<u64>(tab.size());
  if (!d_tab) return fail(c, HE_ENOMEM, "workspace too small for ffconv_layer");
  hipStream_t s = S(stream);
  int e = upload(c, d_tab, tab.data(), tab.size() * 8, s);
  if (e) return e;
  return ffconv_run(c, 1, d_in, 0, level, desc, d_w1_filt, 0, d_mask, d_tab, o_c2, square, d_out, ar, s);
}

int he_int_weight_table(he_ctx* c, const double* h_w, int count, int k_bits, int level, uint64_t* d_tab,
                        void* stream) {
  if (!c || !h_w || !d_tab || count < 1 || k_bits < 0 || k_bits > 40 || !level_ok(c, level))
    return fail(c, HE_EINVAL, "he_int_weight_table: bad arguments");
  std::vector<int64_t> w(count);
  for (int i = 0; i < count; ++i) {
    const double x = std::ldexp(h_w[i], k_bits);
    if (!(std::fabs(x) < 4.0e18)) return fail(c, HE_EINVAL, "he_int_weight_table: weight too large");
    w[i] = round_half_away(x);
  }
  std::vector<u64> tab = scalar_table(c, w, level);
  return upload(c, d_tab, tab.data(), tab.size() * 8, S(stream));
}

int ffconv_layer_batch(he_ctx* c, int n_layers, const uint64_t* d_in, size_t in_stride, int level,
                       const he_conv_desc* desc, const uint64_t* d_w1_filt, size_t filt_stride, const uint64_t* d_mask,
                       const uint64_t* d_w2_tab, int o_c2, int square, uint64_t* d_out, void* stream) {
  if (!c || !d_in || !desc || !d_w1_filt || !d_mask || !d_w2_tab || !d_out || n_layers < 1)
    return fail(c, HE_EINVAL, "ffconv_layer_batch: bad arguments");
  if (o_c2 < 1 || desc->o_c < 1) return fail(c, HE_EINVAL, "ffconv_layer_batch: bad W2 shape");
  if (level < 3 || level > c->big_l) return fail(c, HE_ELEVEL, "ffconv_layer_batch needs level >= 3 (got %d)", level);
  Arena ar(c);
  return ffconv_run(c, n_layers, d_in, in_stride, level, desc, d_w1_filt, filt_stride, d_mask, d_w2_tab, o_c2, square,
                    d_out, ar, S(stream));
}

int he_densepack_hma(he_ctx* c, int n_layers, const uint64_t* d_in, size_t in_stride, int level,
                     const he_conv_desc* desc, const uint64_t* d_filt, size_t filt_stride, uint64_t* d_acc,
                     void* stream) {
  if (!c || !d_in || !desc || !d_filt || !d_acc || n_layers < 1)
    return fail(c, HE_EINVAL, "he_densepack_hma: bad arguments");
  DPGeom geo;
  int n_cls = 0;
  if (!build_geom(c, desc, geo, n_cls)) return fail(c, HE_EINVAL, "he_densepack_hma: bad convolution geometry");
  if (!level_ok(c, level)) return fail(c, HE_ELEVEL, "he_densepack_hma: level %d out of range", level);
  if ((long long)n_layers * geo.per_layer > (1ll << 30)) return fail(c, HE_EINVAL, "he_densepack_hma: too many outputs");
  geo.x_stride = in_stride;
  geo.f_stride = filt_stride;
  const int total = n_layers * geo.per_layer;
  hipStream_t s = S(stream);
  for (int o0 = 0; o0 < total; o0 += 65535) {
    const int cn = std::min(65535, total - o0);
    dispatch_logn<LDpHma>(c->logn, c, d_in, d_filt, d_acc + (size_t)o0 * 2 * level * c->n, level, o0, cn, geo, s);
  }
  c->counts = he_counts{};
  c->counts.mulpc = (int64_t)total * geo.m_cts;
  c->counts.addcc = (int64_t)total * (geo.m_cts - 1);
  return check_launch(c, "he_densepack_hma");
}

int he_rotsum_groups(he_ctx* c, const he_rotsum_group* h_groups, int n_groups, void* stream) {
  if (!c || !h_groups || n_groups < 1) return fail(c, HE_EINVAL, "he_rotsum_groups: bad arguments");
  const int n = c->n;
  size_t total = 0;
  for (int g = 0; g < n_groups; ++g) {
    const he_rotsum_group& gr = h_groups[g];
    if (!gr.acc || gr.count < 0 || !level_ok(c, gr.level) || gr.step < 0 || gr.step > 30)
      return fail(c, HE_EINVAL, "he_rotsum_groups: bad group %d", g);
    if ((1ll << gr.step) % (n / 2) == 0) return fail(c, HE_EINVAL, "he_rotsum_groups: step 2^%d is the identity", gr.step);
    total += (size_t)gr.count;
  }
  if (total == 0) return HE_OK;
  std::vector<KsJob> jobs;
  jobs.reserve(total);
  for (int g = 0; g < n_groups; ++g) {
    const he_rotsum_group& gr = h_groups[g];
    const int k = 1 << gr.step;
    const u32 gal = galois_of(k, n);
    auto it = c->keys.find((int)gal);
    if (it == c->keys.end()) return fail(c, HE_ENOKEY, "he_rotsum_groups: no rotation key for step %d", k);
    const u32 ginv = galois_of(-k, n);
    const size_t cstride = (size_t)2 * gr.level * n;
    for (int i = 0; i < gr.count; ++i) {
      u64* ct = gr.acc + (size_t)i * cstride;
      jobs.push_back(KsJob{ct + (size_t)gr.level * n, ct, ct, it->second, gal, ginv, gr.level, 0});
    }
  }
  Arena ar(c);
  return rotate_jobs(c, jobs, EPI_ROTSUM, ar, S(stream));
}

int ffconv_tail_batch(he_ctx* c, int n_layers, const uint64_t* d_acc, int level, const he_conv_desc* desc,
                      const uint64_t* d_mask, const uint64_t* d_w2_tab, int o_c2, int square, uint64_t* d_out,
                      void* stream) {
  if (!c || !d_acc || !desc || !d_mask || !d_w2_tab || !d_out || n_layers < 1 || o_c2 < 1 || desc->o_c < 1)
    return fail(c, HE_EINVAL, "ffconv_tail_batch: bad arguments");
  const int need = square ? 4 : 3;
  if (level < need || level > c->big_l) return fail(c, HE_ELEVEL, "ffconv_tail_batch needs level >= %d (got %d)", need, level);
  DPGeom geo;
  int n_cls = 0;
  if (!build_geom(c, desc, geo, n_cls)) return fail(c, HE_EINVAL, "ffconv_tail_batch: bad convolution geometry");
  const int r = desc->o_c;
  if ((long long)n_layers * r > 65535 || (long long)n_layers * o_c2 > 65535)
    return fail(c, HE_EINVAL, "ffconv_tail_batch: too many layers for one call");
  if (square && !c->keys.count(0)) return fail(c, HE_ENOKEY, "ffconv_tail_batch: no relinearisation key");
  const int spatial = geo.out_h * geo.out_w;
  const int n = c->n;
  c->counts = he_counts{};
  Arena ar(c);
  hipStream_t s = S(stream);
  const size_t cnt = (size_t)n_layers * r * spatial;
  u64* y = ar.take<u64>(cnt * 2 * (level - 1) * n);
  if (!y) return fail(c, HE_ENOMEM, "workspace too small for ffconv_tail_batch");
  int e = rescale_batch(c, y, d_acc, (int)cnt, level, ar, s);
  c->counts.rescale += (int64_t)cnt;
  if (e) return e;
  return ffconv_tail(c, n_layers, y, level - 1, spatial, r, d_mask, d_w2_tab, o_c2, square, d_out, ar, s);
}

size_t he_ffconv_workspace_need(const he_ctx* c, int n_layers, int level, const he_conv_desc* desc, int o_c2,
                                int square) {
  DPGeom geo;
  int n_cls = 0;
  if (!c || !desc || n_layers < 1 || o_c2 < 1 || level < 3 || level > c->big_l ||
      !build_geom(const_cast<he_ctx*>(c), desc, geo, n_cls))
    return 0;
  return ffconv_need(c, n_layers, level, geo.out_h * geo.out_w, desc->o_c, o_c2, square != 0);
}

// ---- graphs ---------------------------------------------------------------------

int he_graph_begin(he_ctx* c, void* stream) {
  if (!c || !stream) return fail(c, HE_EINVAL, "he_graph_begin: needs a context and a non-default stream");
  if (c->capturing) return fail(c, HE_EINVAL, "he_graph_begin: already capturing");
  if (hipStreamBeginCapture(S(stream), hipStreamCaptureModeThreadLocal) != hipSuccess)
    return fail(c, HE_EDEVICE, "he_graph_begin: hipStreamBeginCapture failed");
  c->capturing = true;
  return HE_OK;
}

int he_graph_end(he_ctx* c, void* stream, he_graph** out) {
  if (!c || !stream || !out) return fail(c, HE_EINVAL, "he_graph_end: bad arguments");
  *out = nullptr;
  if (!c->capturing) return fail(c, HE_EINVAL, "he_graph_end: not capturing");
  c->capturing = false;
  hipGraph_t g = nullptr;
  if (hipStreamEndCapture(S(stream), &g) != hipSuccess || !g)
    return fail(c, HE_EDEVICE, "he_graph_end: capture failed (a call inside it was not capturable)");
  hipGraphExec_t ex = nullptr;
  if (hipGraphInstantiate(&ex, g, nullptr, nullptr, 0) != hipSuccess) {
    (void)hipGraphDestroy(g);
    return fail(c, HE_EDEVICE, "he_graph_end: instantiation failed");
  }
  he_graph* gr = new he_graph();
  gr->ctx = c;
  gr->epoch = c->epoch;
  gr->graph = g;
  gr->exec = ex;
  *out = gr;
  return HE_OK;
}

int he_graph_launch(he_graph* g, void* stream) {
  if (!g || !g->ctx) return HE_EINVAL;
  if (g->epoch != g->ctx->epoch)
    return fail(g->ctx, HE_EINVAL, "he_graph_launch: workspace or keys changed since the capture");
  if (hipGraphLaunch(g->exec, S(stream)) != hipSuccess) return fail(g->ctx, HE_EDEVICE, "hipGraphLaunch failed");
  return HE_OK;
}

int he_graph_destroy(he_graph* g) {
  if (!g) return HE_EINVAL;
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  delete g;
  return HE_OK;
}

int he_prof_select(he_ctx* c, const char* kernel) {
  if (!c) return HE_EINVAL;
  c->prof_kernel = kernel ? kernel : "";
  double ms;
  int64_t n;
  return he_prof_read(c, &ms, &n);
}

int he_prof_read_busy(he_ctx* c, double* total_ms, double* busy_ms, int64_t* launches) {
  if (!c || !total_ms || !busy_ms || !launches) return HE_EINVAL;
  std::vector<std::pair<double, double>> iv;
  double sum = 0;
  if (!c->prof_events.empty()) {
    hipEvent_t ref = c->prof_events.front().first;
    for (auto& pr : c->prof_events) {
      float a = 0, b = 0;
      if (hipEventSynchronize(pr.second) != hipSuccess || hipEventElapsedTime(&a, ref, pr.first) != hipSuccess ||
          hipEventElapsedTime(&b, ref, pr.second) != hipSuccess)
        return fail(c, HE_EDEVICE, "he_prof_read_busy: event failure");
      iv.push_back({a, b});
      sum += b - a;
    }
  }
  std::sort(iv.begin(), iv.end());
  double busy = 0, cs = 0, ce = -1;
  for (auto& x : iv) {
    if (x.first > ce) {
      if (ce > cs) busy += ce - cs;
      cs = x.first;
      ce = x.second;
    } else if (x.second > ce) {
      ce = x.second;
    }
  }
  if (ce > cs) busy += ce - cs;
  *busy_ms = busy;
  double total = 0;
  int64_t n = 0;
  int e = he_prof_read(c, &total, &n);
  *total_ms = sum;
  *launches = n;
  return e;
}

int he_prof_read(he_ctx* c, double* total_ms, int64_t* launches) {
  if (!c || !total_ms || !launches) return HE_EINVAL;
  double sum = 0;
  for (auto& pr : c->prof_events) {
    float ms = 0;
    if (hipEventSynchronize(pr.second) != hipSuccess || hipEventElapsedTime(&ms, pr.first, pr.second) != hipSuccess)
      return fail(c, HE_EDEVICE, "he_prof_read: event failure");
    sum += ms;
    c->prof_pool.push_back(pr.first);
    c->prof_pool.push_back(pr.second);
  }
  *total_ms = sum;
  *launches = (int64_t)c->prof_events.size();
  c->prof_events.clear();
  return HE_OK;
}

int he_last_counts(const he_ctx* c, he_counts* out) {
  if (!c || !out) return HE_EINVAL;
  *out = c->counts;
  return HE_OK;
}

}  // extern "C"

// Internal state of a library context and the launch wrappers shared by the
// C-ABI unit (capi.hip) and the per-ring-size launch units (launch_n*.hip,
// which instantiate the kernels of one log2 N each, so the library builds in
// parallel).  Not part of the public interface.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdio>
#include <map>
#include <string>
#include <vector>

#include "../../include/ffconv_he.h"
#include "host_params.h"
#include "kernels.h"

namespace he {
// Pinned staging ring for small host tables (job tables, weight residues).
struct StageSlot {
  char* host = nullptr;
  size_t cap = 0;
  hipEvent_t ev = nullptr;
  bool pending = false;
};
constexpr int STAGE_SLOTS = 64;
}  // namespace he

using namespace he;

// Most chains (one stream each) a DensePack rotate-and-sum is split into.
constexpr int MAX_SPLIT = 4;

struct he_ctx {
  int n = 0, logn = 0, big_l = 0;
  std::vector<u64> moduli;  // q_0..q_{L-1}, P
  Mods mods{};
  bool has_cls[3] = {false, false, false};  // width classes among q_0..q_{L-1}, P
  unsigned q_mask = 0;                       // bit c: a ciphertext prime of class c exists
  int p_cls = 0;                             // class of P
  u64* d_tw = nullptr;    // [L+1][4][N] 64-bit twiddles + Shoup companions
  u32* d_tw32 = nullptr;  // 32-bit copies for the narrow moduli
  double* d_twf = nullptr;  // (w, w / q) as doubles for the f64 moduli
  // forward twiddles of the two half-ring transforms that follow a transform's
  // first stage, [L+1][2 halves][2 (w, companion)][N/2], in the three word types
  u64* d_twh = nullptr;
  u32* d_twh32 = nullptr;
  double* d_twhf = nullptr;
  u64* d_inv = nullptr;   // [2][HE_MAXM][HE_MAXM]: m_div^-1 mod q_t and Shoup components
  Tables tb() const { return Tables{d_tw, d_tw32, d_twf, d_twh, d_twh32, d_twhf}; }
  int pg_set[HE_MAXM + 1] = {};  // P groups per key-switch level (0 = cost model)
  int split_streams = 1;         // DensePack rotate-and-sum split over several streams
  int split_parts = 2;           // ... into this many chains (2..MAX_SPLIT), one stream each
  int moddown_halves = -1;       // ModDown as two half-ring workgroups per limb (-1: from N = 16384)
  int hoist_fused = 0;           // hoisted rotations: ModDown fused with the inner product (measured slower)
  int hoist_pipeline = 0;        // hoisted rotations: inner products and ModDown of chunks on two streams (slower)
  // ModUp as two half-ring workgroups per target, per key-switch level
  // (-1: by ring size)
  int halves_set[HE_MAXM + 1] = {-1, -1, -1, -1, -1, -1, -1, -1, -1, -1, -1, -1, -1, -1, -1, -1, -1};
  char* ws = nullptr;
  size_t ws_bytes = 0;
  bool ws_owned = true;  // false: the caller's buffer (he_ctx_set_workspace)
  char* fixed_scratch = nullptr;  // this device's static scratch array (he_rotate_static)
  std::map<int, u64*> keys;  // Galois element (0 = relinearisation) -> [L][2][L+1][N]
  std::string err;
  he_counts counts{};
  int device = 0;
  // instrumentation: events around launches of one selected kernel
  std::string prof_kernel;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> prof_events;
  std::vector<hipEvent_t> prof_pool;
  // second stream (default priority) for the other width classes of a launch
  hipStream_t side = nullptr;
  hipEvent_t fork_ev = nullptr, join_ev = nullptr;
  // further streams (default priority) and their join events for a DensePack
  // rotate-and-sum split into up to MAX_SPLIT chains
  hipStream_t side_x[MAX_SPLIT - 2] = {};
  hipEvent_t join_x[MAX_SPLIT - 2] = {};
  hipEvent_t pipe_ev[4] = {};  // one per chunk of a hoisted-rotation pipeline
  StageSlot stage[STAGE_SLOTS];
  int stage_next = 0;
  // graph capture: set between he_graph_begin and he_graph_end; epoch counts
  // changes that move memory a captured graph refers to (workspace, keys)
  bool capturing = false;
  uint64_t epoch = 0;
};

struct he_graph {
  he_ctx* ctx = nullptr;
  uint64_t epoch = 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace he {

inline int fail(he_ctx* c, int code, const char* fmt, ...) {
  if (c) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    c->err = buf;
  }
  return code;
}

inline int check_launch(he_ctx* c, const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(c, HE_EDEVICE, "%s: %s", what, hipGetErrorString(e));
  return HE_OK;
}

inline hipStream_t S(void* s) { return (hipStream_t)s; }

inline hipEvent_t prof_event(he_ctx* c) {
  if (!c->prof_pool.empty()) {
    hipEvent_t e = c->prof_pool.back();
    c->prof_pool.pop_back();
    return e;
  }
  // timing only: these events order no data (their pairs are read after the
  // stream has been synchronised), so they skip the system-scope fence and
  // its cache write-back between the kernels they bracket
  hipEvent_t e = nullptr;
  if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) return nullptr;
  return e;
}

// Brackets the launches in its scope with events when `name` is selected.
struct Prof {
  he_ctx* c;
  hipStream_t s;
  hipEvent_t a = nullptr;
  Prof(he_ctx* ctx, const char* name, hipStream_t st) : c(ctx), s(st) {
    if (!c->capturing && !c->prof_kernel.empty() && c->prof_kernel == name) {
      a = prof_event(c);
      if (a) (void)hipEventRecord(a, s);
    }
  }
  ~Prof() {
    if (!a) return;
    hipEvent_t b = prof_event(c);
    if (!b) return;
    (void)hipEventRecord(b, s);
    c->prof_events.push_back({a, b});
  }
};

// Bump allocator over the context workspace (one per call).
struct Arena {
  char* base;
  size_t cap, used = 0;
  Arena(he_ctx* c) : base(c->ws), cap(c->ws_bytes) {}
  Arena(char* b, size_t bytes) : base(b), cap(bytes) {}
  template <typename T>
  T* take(size_t count) {
    size_t bytes = (count * sizeof(T) + 255) & ~(size_t)255;
    if (used + bytes > cap) return nullptr;
    T* p = (T*)(base + used);
    used += bytes;
    return p;
  }
  size_t left() const { return cap - used; }
  // The remaining space split into k disjoint arenas of about 1/k each.
  void split(int k, Arena* out) const {
    const size_t part = (left() / (size_t)k) & ~(size_t)255;
    for (int i = 0; i < k; ++i) {
      out[i] = *this;
      out[i].used = used + (size_t)i * part;
      out[i].cap = (i == k - 1) ? cap : used + (size_t)(i + 1) * part;
    }
  }
};

inline u32 galois_of(int k, int n) {
  const int slots = n / 2;
  int e = k % slots;
  if (e < 0) e += slots;
  return (u32)powmod(5, (u64)e, 2 * (u64)n);
}

template <template <int> class F, typename... A>
inline int dispatch_logn(int logn, A&&... args) {
  switch (logn) {
    case 10: F<10>::run(args...); return 0;
    case 11: F<11>::run(args...); return 0;
    case 12: F<12>::run(args...); return 0;
    case 13: F<13>::run(args...); return 0;
    case 14: F<14>::run(args...); return 0;
    default: return -1;
  }
}

// Runs LAUNCH with the constant CLS bound to every width class in `mask`
// (transform kernels are instantiated per class).
#define HE_FOR_CLASSES(mask, LAUNCH)               \
  do {                                             \
    if ((mask)&1u) {                               \
      constexpr int CLS = CLS_N32;                 \
      LAUNCH;                                      \
    }                                              \
    if ((mask)&2u) {                               \
      constexpr int CLS = CLS_F64;                 \
      LAUNCH;                                      \
    }                                              \
    if ((mask)&4u) {                               \
      constexpr int CLS = CLS_U64;                 \
      LAUNCH;                                      \
    }                                              \
  } while (0)

inline unsigned cls_mask(const he_ctx* c, int first, int count) {
  unsigned m = 0;
  for (int i = first; i < first + count; ++i) m |= 1u << c->mods.m[i].cls;
  return m;
}

// ---- launch wrappers (templated on log2 N; defined in launch.h and
// instantiated for N = 2^10 .. 2^14 in launch_n10.hip .. launch_n14.hip) ----
template <int LOGN>
struct LNtt {
  static void run(he_ctx* c, u64* d, int n_polys, int n_limbs, int first_mod, bool fwd, hipStream_t s);
};
template <int LOGN>
struct LKsCore {
  static void run(he_ctx* c, const KsJob* jobs, int count, int lmax, int pg, u64* dcoef, u64* u, u64* rc,
                  hipStream_t s, int pk = 0, bool digits_done = false);
};
template <int LOGN>
struct LDrop {
  static void run(he_ctx* c, int mode, int epi, const KsJob* jobs, int count, int lmax, int urows, const u64* u,
                  const u64* rc, hipStream_t s, int pk = 0, NextDigits nd = NextDigits{nullptr, 1u, 0});
};
template <int LOGN>
struct LIntt1 {
  static void run(he_ctx* c, const KsJob* jobs, int count, int lmax, u64* rc, hipStream_t s, int pk = 0);
};
template <int LOGN>
struct LDpHma {
  static void run(he_ctx* c, const u64* x, const u64* filt, u64* out, int level, int out_base, int n_out,
                  const DPGeom& geo, hipStream_t s, bool out_packed = false);
};
template <int LOGN>
struct LHmaPerm {
  static void run(he_ctx* c, u64* acc, const u64* cts, int K, const u64* pts, int pt_stride, int pt_limbs,
                  const int32_t* gal, u32 g_step, int level, int accumulate, int n_acc, hipStream_t s);
};
template <int LOGN>
struct LKeygen {
  static void run(he_ctx* c, u64* key, const u64* sk, const u64* a, const u64* ehat, u32 g, ConstTable pm,
                  hipStream_t s, int pack);
};
template <int LOGN>
struct LHoistUp {
  static void run(he_ctx* c, const KsJob* jobs1, int count, int level, u64* dcoef, u64* dhat, hipStream_t s);
};
template <int LOGN>
struct LHoisted {
  // part: 0 all, 1 the inner products only, 2 the P INTT and ModDown only;
  // add_c0 (with part 1): the inner products also get P sigma_g(c0)
  static void run(he_ctx* c, const KsJob* jobs, int m, int level, const u64* dhat, u64* u, u64* rc, hipStream_t s,
                  int job_base = 0, int per_ct = 1 << 30, size_t dstride = 0, int part = 0, int add_c0 = 0);
};
struct TapMap;
template <int LOGN>
struct LModDown {  // P INTT + ModDown (store) of count key-switch row sets u [2][level + 1][N]
  static void run(he_ctx* c, const KsJob* jobs, int count, int level, const u64* u, u64* rc, hipStream_t s);
};
template <int LOGN>
struct LTapHmaQp {
  static void run(he_ctx* c, const u64* x, const u64* u, const u64* filt, const u64* fp, u64* out, int level,
                  int pt_limbs, const TapMap& tm, int n_b, hipStream_t s);
};
template <int LOGN>
struct LTapHma {
  static void run(he_ctx* c, const u64* x, const u64* rot, const u64* filt, u64* out, int level, int pt_limbs,
                  const TapMap& tm, int n_b, hipStream_t s);
};

}  // namespace he

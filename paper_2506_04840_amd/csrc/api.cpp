// C ABI front end: argument checks, workspace carving and the launch sequence of
// shifted randomized T-HOSVD (Algorithm 2) and ST-HOSVD (Algorithm 3).
// Every call validates on the host first and either enqueues all its work on
// the caller's stream or returns an error having enqueued nothing. Nothing
// here waits on the device: the shift branch runs in a kernel, so a whole
// solve is one stream of launches.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "internal.hpp"
#include "tucker.h"

using namespace tk;

namespace {

thread_local std::string g_err_text;
thread_local int g_err_code = 0;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err_text = buf;
  g_err_code = code;
  return code;
}

int dev_check(hipError_t e, const char* what) {
  if (e != hipSuccess) return fail(TUCKER_EDEVICE, "%s: %s", what, hipGetErrorString(e));
  return TUCKER_OK;
}

bool valid_prec(int p) { return p == TUCKER_FP64 || p == TUCKER_FP32 || p == TUCKER_BF16; }

// Checks a shape; fills numel. Returns 0 or an error code (with detail).
int check_shape(const tucker_shape* s, int64_t* numel) {
  if (s == nullptr) return fail(TUCKER_EINVAL, "shape is null");
  if (s->order < 1 || s->order > TUCKER_MAX_ORDER)
    return fail(TUCKER_EINVAL, "order %d outside 1..%d", s->order, TUCKER_MAX_ORDER);
  int64_t n = 1;
  for (int k = 0; k < s->order; ++k) {
    if (s->dims[k] < 1) return fail(TUCKER_EINVAL, "dims[%d] = %lld < 1", k, (long long)s->dims[k]);
    if (n > ((int64_t)1 << 62) / s->dims[k]) return fail(TUCKER_EINVAL, "tensor size overflows int64");
    n *= s->dims[k];
  }
  *numel = n;
  return TUCKER_OK;
}

View3 view_of(const int64_t* dims, int d, int k) {
  View3 v{1, dims[k], 1};
  for (int j = 0; j < k; ++j) v.P *= dims[j];
  for (int j = k + 1; j < d; ++j) v.S *= dims[j];
  return v;
}

struct Plan {
  int d;
  int64_t dims[TUCKER_MAX_ORDER];
  int64_t r[TUCKER_MAX_ORDER];
  int ord[TUCKER_MAX_ORDER];  // processing order: ord[i] is the i-th mode processed
  int l[TUCKER_MAX_ORDER];
  int64_t m[TUCKER_MAX_ORDER];
  View3 v[TUCKER_MAX_ORDER];  // view of the tensor each mode's products read
  bool st;
  bool holistic;        // Appendix A / B variants: modes keep width l_k, then a small HOSVD
  bool one_stream = false;  // every launch on the caller's stream (no side stream for the small SVDs)
  int32_t flags;
  int64_t xbuf_elems;   // largest intermediate of the core chain
  int64_t omz_elems;    // largest m_k * l_k (Omega / Z)
  int64_t nl_max;       // largest n_k * l_k
  int64_t n_max;
  int l_max;
  size_t part_bytes;
  size_t orth_bytes;
  // holistic variants: the small tensor B (sizes l_k) and its deterministic HOSVD
  int64_t b_elems;      // numel(B)
  size_t orth2_bytes;   // largest orthonormalisation workspace of phase 2
  int64_t napart_elems; // ||A||^2 partial sums of the first mode's sketch (or of the plain norm pass)
};

// Processing order of an options struct (nullptr: natural) into ord[0..d-1].
int resolve_order(const tucker_options* opt, int d, const int64_t* dims, int* ord) {
  for (int i = 0; i < d; ++i) ord[i] = i;
  if (opt == nullptr || opt->order_kind == TUCKER_ORDER_NATURAL) return TUCKER_OK;
  if (opt->order_kind == TUCKER_ORDER_DECREASING) {
    // stable: equal sizes keep increasing mode order
    std::stable_sort(ord, ord + d, [&](int a, int b) { return dims[a] > dims[b]; });
    return TUCKER_OK;
  }
  if (opt->order_kind != TUCKER_ORDER_GIVEN) return fail(TUCKER_EINVAL, "unknown order kind %d", opt->order_kind);
  bool seen[TUCKER_MAX_ORDER] = {};
  for (int i = 0; i < d; ++i) {
    const int k = opt->order[i];
    if (k < 0 || k >= d || seen[k])
      return fail(TUCKER_EINVAL, "order[0..%d] is not a permutation of 0..%d", d - 1, d - 1);
    seen[k] = true;
    ord[i] = k;
  }
  for (int i = d; i < TUCKER_MAX_ORDER; ++i)
    if (opt->order[i] != 0) return fail(TUCKER_EINVAL, "order[%d] beyond the tensor order is not zero", i);
  return TUCKER_OK;
}

int make_plan(const tucker_shape* shape, const int64_t* ranks, int32_t p, int32_t q, tucker_precision prec,
              bool st, Plan* pl, const tucker_options* opt = nullptr) {
  int64_t numel;
  int rc = check_shape(shape, &numel);
  if (rc) return rc;
  if (ranks == nullptr) return fail(TUCKER_EINVAL, "ranks is null");
  if (p < 0) return fail(TUCKER_EINVAL, "oversampling p = %d < 0", p);
  if (q < 0 || q > TUCKER_MAX_Q) return fail(TUCKER_EINVAL, "power count q = %d outside 0..%d", q, TUCKER_MAX_Q);
  if (!valid_prec(prec)) return fail(TUCKER_EINVAL, "bad precision %d", (int)prec);
  const int d = shape->order;
  pl->d = d;
  pl->st = st;
  pl->holistic = opt != nullptr && opt->holistic != 0;
  pl->flags = 0;
  int64_t cur[TUCKER_MAX_ORDER];
  for (int k = 0; k < d; ++k) {
    pl->dims[k] = shape->dims[k];
    cur[k] = shape->dims[k];
    pl->r[k] = ranks[k];
    if (ranks[k] < 1 || ranks[k] > shape->dims[k])
      return fail(TUCKER_EINVAL, "rank r[%d] = %lld outside 1..n[%d] = %lld", k, (long long)ranks[k], k,
                  (long long)shape->dims[k]);
  }
  pl->xbuf_elems = 1;
  pl->omz_elems = 1;
  pl->nl_max = 1;
  pl->n_max = 1;
  pl->l_max = 1;
  pl->part_bytes = 256;
  pl->orth_bytes = 256;
  rc = resolve_order(opt, d, pl->dims, pl->ord);
  if (rc) return rc;
  // per-mode fields are indexed by mode; ST-HOSVD's sizes follow the order
  for (int i = 0; i < d; ++i) {
    const int k = pl->ord[i];
    const int64_t* src = st ? cur : pl->dims;
    int64_t nk = src[k], mk = 1;
    for (int j = 0; j < d; ++j)
      if (j != k) mk *= src[j];
    if (pl->r[k] > mk)
      return fail(TUCKER_EINVAL,
                  "rank r[%d] = %lld exceeds the other modes' product m = %lld (no unfolding has that rank)", k,
                  (long long)pl->r[k], (long long)mk);
    const int64_t lk = std::min<int64_t>(std::min<int64_t>(pl->r[k] + p, nk), mk);
    if (lk > TUCKER_MAX_L)
      return fail(TUCKER_EUNSUPPORTED, "sketch width l[%d] = %lld exceeds %d", k, (long long)lk, TUCKER_MAX_L);
    if (lk < pl->r[k] + p) pl->flags |= TUCKER_INFO_L_CLAMPED;
    pl->l[k] = (int)lk;
    pl->m[k] = mk;
    pl->v[k] = view_of(src, d, k);
    pl->omz_elems = std::max(pl->omz_elems, mk * lk);
    pl->nl_max = std::max(pl->nl_max, nk * lk);
    pl->n_max = std::max(pl->n_max, nk);
    pl->l_max = std::max(pl->l_max, (int)lk);
    pl->part_bytes = std::max(pl->part_bytes, colreduce_part_bytes(pl->v[k], (int)lk, prec));
    pl->orth_bytes = std::max(pl->orth_bytes, orth_ws_bytes(nk, (int)lk));
    if (st) cur[k] = pl->holistic ? lk : pl->r[k];
  }
  // core chain intermediates: ST contracts in processing order, T in mode order
  // (the holistic variants keep l_k columns there)
  int64_t chain[TUCKER_MAX_ORDER];
  for (int k = 0; k < d; ++k) chain[k] = pl->dims[k];
  for (int i = 0; i + 1 < d; ++i) {
    const int k = st ? pl->ord[i] : i;
    chain[k] = pl->holistic ? pl->l[k] : pl->r[k];
    int64_t e = 1;
    for (int j = 0; j < d; ++j) e *= chain[j];
    pl->xbuf_elems = std::max(pl->xbuf_elems, e);
  }
  // ||A||^2 rides on the sketch of the first mode processed (every element of
  // A is staged once there), or takes its own pass when that mode has S == 1
  {
    const int k0 = pl->ord[0];
    const int64_t slots = colreduce_norm_slots(pl->v[k0], colreduce_splits(pl->v[k0], pl->l[k0]));
    pl->napart_elems = std::max<int64_t>(std::max<int64_t>(slots, norm2_blocks(numel)), 1);
  }
  pl->b_elems = 1;
  pl->orth2_bytes = 256;
  if (pl->holistic && d < 2) return fail(TUCKER_EUNSUPPORTED, "the holistic variants need order d >= 2");
  if (pl->holistic) {
    // phase 2 walks the small tensor: mode k's unfolding is l_k x m with m the
    // product of the other current sizes (ST: r for the modes done, l else)
    int64_t c2[TUCKER_MAX_ORDER];
    for (int k = 0; k < d; ++k) {
      c2[k] = pl->l[k];
      pl->b_elems *= pl->l[k];
    }
    for (int i = 0; i < d; ++i) {
      const int k = pl->ord[i];
      int64_t m = 1;
      for (int j = 0; j < d; ++j)
        if (j != k) m *= c2[j];
      if (pl->r[k] > m)
        return fail(TUCKER_EINVAL, "rank r[%d] = %lld exceeds the small tensor's other sizes' product %lld", k,
                    (long long)pl->r[k], (long long)m);
      const int64_t lk = pl->l[k];
      pl->orth2_bytes = std::max(pl->orth2_bytes, m >= lk ? orth_ws_bytes(m, (int)lk) : orth_ws_bytes(lk, (int)m));
      if (st) c2[k] = pl->r[k];
    }
  }
  return TUCKER_OK;
}

struct ModeWs {
  void* omz;
  void* part;
  double* y64;
  void* qt;
  void* ut;
  double* q64;
  double* sigma;
  void* orth;
  double* sig_hat;
  int* stop;
};

struct SolveWs {
  void* xbuf[2];
  void* omz;
  void* part;
  double* y64;
  void* qt;    // Q j-major (l x n), storage precision: the power step's X^T Q operand
  void* ut;    // U_k j-major (r x n), storage precision: the core step's operand
  double* q64;
  double* sigma;
  double* alpha;
  double* normpart;
  void* orth;
  double* sig_hat;  // per-vector-error estimates of the previous step (Algorithm 4)
  int* stop;        // its stopping flag
  double* napart;   // ||A||^2 partial sums
  double* na2;      // where the mode that carries ||A||^2 writes it (nullptr in the other modes)
  ModeWs mode_store[TUCKER_MAX_ORDER];
  ModeWs* mode[TUCKER_MAX_ORDER];  // T-HOSVD: own scratch of modes 1..d-1 (else nullptr)
  // holistic variants
  double* hq64[TUCKER_MAX_ORDER];  // Q_k, n_k x l_k FP64
  void* hqt[TUCKER_MAX_ORDER];     // Q_k^T j-major (l_k x n_k), storage precision
  void* hvt[TUCKER_MAX_ORDER];     // signed V_k^T j-major (r_k x l_k), storage precision
  void* bbuf;                      // the small tensor B
  double* y2;                      // phase-2 unfolding, FP64
  void* orth2;
  double* v2;                      // phase-2 singular vectors (l_k x l_k at most)
  double* sig2;

  // the scratch mode k works in (shared pointers stay)
  SolveWs for_mode(int k) const {
    SolveWs c = *this;
    if (k >= 0 && k < TUCKER_MAX_ORDER && mode[k] != nullptr) {
      const ModeWs& m = *mode[k];
      c.omz = m.omz;
      c.part = m.part;
      c.y64 = m.y64;
      c.qt = m.qt;
      c.ut = m.ut;
      c.q64 = m.q64;
      c.sigma = m.sigma;
      c.orth = m.orth;
      c.sig_hat = m.sig_hat;
      c.stop = m.stop;
    }
    return c;
  }
};

size_t solve_ws_layout(const Plan& pl, tucker_precision prec, char* base, SolveWs* w) {
  const size_t es = elem_bytes(prec);
  size_t off = 0;
  auto take = [&](size_t bytes) -> void* {
    void* p = base ? base + off : nullptr;
    off += align_up(bytes);
    return p;
  };
  w->xbuf[0] = take((size_t)pl.xbuf_elems * es);
  w->xbuf[1] = take((size_t)pl.xbuf_elems * es);
  w->omz = take((size_t)pl.omz_elems * es);
  w->part = take(pl.part_bytes);
  w->y64 = (double*)take((size_t)pl.nl_max * 8);
  w->qt = take((size_t)pl.nl_max * es);
  w->ut = take((size_t)pl.nl_max * es);
  w->q64 = (double*)take((size_t)pl.nl_max * 8);
  w->sigma = (double*)take(TUCKER_MAX_L * 8);
  w->alpha = (double*)take(TUCKER_MAX_ORDER * 8);
  w->normpart = (double*)take(1024 * 8);
  w->orth = take(pl.orth_bytes);
  w->sig_hat = (double*)take(TUCKER_MAX_L * 8);
  w->stop = (int*)take(64);
  w->napart = (double*)take((size_t)pl.napart_elems * 8);
  w->na2 = nullptr;
  // T-HOSVD: the modes are independent and run concurrently; modes 1..d-1
  // get their own copy of the per-mode scratch (mode 0 uses the one above)
  for (int k = 0; k < TUCKER_MAX_ORDER; ++k) {
    w->mode[k] = nullptr;
    w->hq64[k] = nullptr;
    w->hqt[k] = w->hvt[k] = nullptr;
  }
  w->bbuf = w->orth2 = nullptr;
  w->y2 = w->v2 = w->sig2 = nullptr;
  if (pl.holistic) {
    const size_t cs = elem_bytes(prec == TUCKER_BF16 ? TUCKER_FP32 : prec);  // core-chain storage
    for (int k = 0; k < pl.d; ++k) {
      w->hq64[k] = (double*)take((size_t)pl.dims[k] * pl.l[k] * 8);
      w->hqt[k] = take((size_t)pl.dims[k] * pl.l[k] * cs);
      w->hvt[k] = take((size_t)pl.r[k] * pl.l[k] * cs);
    }
    w->bbuf = take((size_t)pl.b_elems * cs);
    w->y2 = (double*)take((size_t)pl.b_elems * 8);
    w->orth2 = take(pl.orth2_bytes);
    w->v2 = (double*)take(TUCKER_MAX_L * TUCKER_MAX_L * 8);
    w->sig2 = (double*)take(TUCKER_MAX_L * 8);
  }
  if (!pl.st && !pl.holistic)
    for (int k = 1; k < pl.d; ++k) {
      ModeWs& mw = w->mode_store[k];
      mw.omz = take((size_t)pl.omz_elems * es);
      mw.part = take(pl.part_bytes);
      mw.y64 = (double*)take((size_t)pl.nl_max * 8);
      mw.qt = take((size_t)pl.nl_max * es);
      mw.ut = take((size_t)pl.nl_max * es);
      mw.q64 = (double*)take((size_t)pl.nl_max * 8);
      mw.sigma = (double*)take(TUCKER_MAX_L * 8);
      mw.orth = take(pl.orth_bytes);
      mw.sig_hat = (double*)take(TUCKER_MAX_L * 8);
      mw.stop = (int*)take(64);
      w->mode[k] = &mw;
    }
  return off;
}

uint64_t completion_seed(uint64_t seed, int mode) {
  return (seed ^ 0x6A09E667F3BCC909ull) * 0x9E3779B97F4A7C15ull + (uint64_t)(mode + 1);
}

// Side stream for the small SVDs of the intermediate iterates (one per host
// thread and device, default priority, created on first use). The SVD of
// step t only feeds step t + 1 through alpha_t and the basis change Wm, both
// applied after step t + 1's two tensor products, so those products run on
// the caller's stream while the SVD runs beside them.
struct SideCtx {
  int dev = -1;
  hipStream_t s = nullptr;
  hipEvent_t qr_done = nullptr, svd_done = nullptr;
  hipStream_t ms = nullptr;  // the mode's own stream (concurrent T-HOSVD modes 1..d-1)
  hipEvent_t fork = nullptr, join = nullptr;
  // the sketch's small SVD when power steps follow (it only feeds the logs)
  hipStream_t ls = nullptr;
  hipEvent_t log_fork = nullptr, log_done = nullptr;
};
thread_local SideCtx g_side[16][TUCKER_MAX_ORDER];

// Streams and events of lane `lane` (a mode of a concurrent T-HOSVD; lane 0
// otherwise), created on first use per host thread and device, default priority.
int side_ctx(SideCtx** out, int lane = 0) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return dev_check(e, "hipGetDevice");
  if (dev < 0 || dev >= 16) return fail(TUCKER_EDEVICE, "device ordinal %d outside 0..15", dev);
  if (lane < 0 || lane >= TUCKER_MAX_ORDER) return fail(TUCKER_EINVAL, "internal: lane %d", lane);
  SideCtx& c = g_side[dev][lane];
  if (c.s == nullptr) {
    e = hipStreamCreateWithFlags(&c.s, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&c.qr_done, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&c.svd_done, hipEventDisableTiming);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&c.ms, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&c.fork, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&c.join, hipEventDisableTiming);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&c.ls, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&c.log_fork, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&c.log_done, hipEventDisableTiming);
    if (e != hipSuccess) return dev_check(e, "side stream setup");
    c.dev = dev;
  }
  *out = &c;
  return TUCKER_OK;
}

// Scratch of tucker_rsthosvd_noalloc: one array per device, part of the
// library's code object, so that entry point never allocates. In host code
// `scratch` names a host-side stand-in, not the device array: the device
// address comes from hipGetSymbolAddress, once per device with that device
// current, and only that address is ever handed to kernels.
static __device__ __align__(256) unsigned char scratch[TUCKER_NOALLOC_SCRATCH_BYTES];
void* g_scratch_addr[16] = {};
std::mutex g_scratch_mu;

int noalloc_scratch(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return dev_check(e, "hipGetDevice");
  if (dev < 0 || dev >= 16) return fail(TUCKER_EDEVICE, "device ordinal %d outside 0..15", dev);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_addr[dev] == nullptr) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return dev_check(e, "hipGetSymbolAddress(scratch)");
    if (p == nullptr) return fail(TUCKER_EDEVICE, "hipGetSymbolAddress(scratch) returned a null address");
    g_scratch_addr[dev] = p;
  }
  *out = g_scratch_addr[dev];
  return TUCKER_OK;
}

// ||A||^2 into *w.na2 for the mode that carries it, right after its sketch:
// the fixed-order sum of the partials that sketch wrote (S > 1), or a pass of
// its own over X (S == 1, whose column reduction stages no rows).
hipError_t launch_norm_of_input(tucker_precision prec, const View3& v, const void* X, int nsplit, const SolveWs& w,
                                hipStream_t st) {
  if (v.S > 1) return launch_norm2_final(w.napart, colreduce_norm_slots(v, nsplit), w.na2, st);
  return launch_norm2(prec, X, v.P * v.n * v.S, w.napart, w.na2, st);
}

// Element count of a mode's tensor from which step 1 rotates its iterate by
// the sketch's J (see mode_factor): a power step over 2^28 elements takes
// about half a millisecond or more, the sketch's small SVD at l <= 64 less.
constexpr double kRotateStep1Numel = 268435456.0;

// One mode of Algorithm 2 / 3 up to U_k (before truncation):
//   Y = X_(k) Omega_k; [Q, Sigma] = svd(Y); alpha_0 = 0;
//   q times: Y = X_(k) (X_(k)^T Q) - alpha Q; [Q, Sigma] = svd(Y); shift update.
// Each svd is split into its CholeskyQR part (Y = Q3 R, on the caller's
// stream) and the small SVD R = J Sigma V^T (side stream except for the last
// one). Step t + 1 runs its products on Q3 instead of Q = Q3 J; the reduce
// subtracts alpha_t Q3 and the next Gram kernel applies J: (X X^T Q3 -
// alpha Q3) J = X X^T Q - alpha Q, the same iterate. Step 1 does not wait
// for the sketch's SVD (alpha_0 = 0 and J_0 does not change the iterate's
// left singular vectors): in modes whose products are short, that SVD no
// longer sits on the critical path. In modes of at least kRotateStep1Numel
// elements it does apply J_0, after the products. On return ws.q64 holds the
// left singular vectors of the last iterate (FP64, n x l, descending).
int mode_factor(const Plan& pl, int k, const void* X, int q, tucker_shift shift, uint64_t seed, tucker_precision prec,
                tucker_info* info, const SolveWs& w, hipStream_t st, const OmegaSpec& om, int lane = 0,
                void* qt_out = nullptr) {
  const View3 v = pl.v[k];
  const int l = pl.l[k];
  const int64_t n = v.n, m = pl.m[k];
  const int nsplit = colreduce_splits_for(v, l, prec);
  const OrthWs ows = carve_orth(w.orth, n, l);
  const uint64_t cseed = completion_seed(seed, k);
  double* alpha = w.alpha + k;
  double* alpha_upd = shift == TUCKER_SHIFT_ADAPTIVE ? alpha : nullptr;
  SideCtx* side = nullptr;
  if (q > 0 && !pl.one_stream) {
    const int rc = side_ctx(&side, lane);
    if (rc) return rc;
  }
  // the small SVDs of steps 0..q-1 run on the side stream, or in line on the
  // caller's stream when the plan asks for one stream (same kernels, same order
  // of dependent work, so the same results)
  const hipStream_t svd_s = side != nullptr ? side->s : st;
  // BF16 operands: the products of the last step (the sketch when q = 0) run
  // on FP32 operands, with FP32 orthonormalisation settings, so the final
  // subspace carries FP32 rather than BF16 rounding (storage is FP32 either way)
  auto step_prec = [&](int t) { return prec == TUCKER_BF16 && t == q ? TUCKER_FP32 : prec; };
  hipError_t e;
  // sketch: Y = X_(k) Omega_k, then its CholeskyQR
  e = launch_fill_omega(om, prec == TUCKER_FP64 ? TUCKER_FP64 : TUCKER_FP32, seed, (uint32_t)k, 0, m, l, true, w.omz,
                        st);
  if (e == hipSuccess)
    e = launch_colreduce(step_prec(0), v, X, w.omz, l, w.part, nsplit, st, w.na2 != nullptr ? w.napart : nullptr);
  if (e == hipSuccess && w.na2 != nullptr) e = launch_norm_of_input(prec, v, X, nsplit, w, st);
  if (e == hipSuccess)
    e = launch_reduce_splits(step_prec(0), w.part, nsplit, n * l, nullptr, prec, nullptr, w.y64, st);
  if (e == hipSuccess) e = launch_mode_start(alpha, ows.pf_ctr, st);
  int nfused = 0;  // fused power steps launched since the counter was zeroed
  // With power steps to follow, the sketch's small SVD feeds only the logs
  // (alpha_0 = 0, and step 1 factors the unrotated iterate): on a stream of
  // its own, with its own R set and Wm, it runs beside the whole power
  // iteration and is joined back at the end of the mode.
  const bool log_sketch = q > 0 && side != nullptr;
  const OrthWs ows0 = log_sketch ? orth_log_set(ows) : orth_step_set(ows, 0);
  // Step 1 factors the unrotated iterate, so that it need not wait for the
  // sketch's SVD; its own SVD then starts from a dense R (about 0.5 ms at
  // l = 60, against 0.13 ms from a rotated iterate). In a mode whose products
  // take longer than the sketch's SVD, step 1 waits for that SVD after its
  // products and rotates its iterate by the sketch's J like every later step
  // (the wait is hidden behind the products, and step 1's SVD starts from a
  // nearly diagonal R).
  const bool rot1 = log_sketch && (double)v.P * (double)v.n * (double)v.S >= kRotateStep1Numel;
  if (e == hipSuccess) e = launch_orth_qr(n, l, w.y64, nullptr, step_prec(0), w.qt, ows0, cseed, 0, st);
  if (e == hipSuccess && log_sketch) {
    e = hipEventRecord(side->log_fork, st);
    if (e == hipSuccess) e = hipStreamWaitEvent(side->ls, side->log_fork, 0);
    if (e == hipSuccess) e = launch_orth_svd(l, step_prec(0), ows0, nullptr, nullptr, info, k, 0, side->ls, nullptr,
                                             nullptr, /*last=*/false);
    if (e == hipSuccess) e = hipEventRecord(side->log_done, side->ls);
  }
  for (int t = 1; t <= q && e == hipSuccess; ++t) {
    const tucker_precision tp = step_prec(t);
    // small SVD of step t - 1 beside the products of step t (each step's R,
    // flags and status in the set of its parity, so step t factors while the
    // SVD of step t - 1 still reads its own)
    const bool svd_prev = !(t == 1 && log_sketch);
    if (svd_prev && side != nullptr) {
      e = hipEventRecord(side->qr_done, st);
      if (e == hipSuccess) e = hipStreamWaitEvent(side->s, side->qr_done, 0);
    }
    if (e == hipSuccess && svd_prev)
      e = launch_orth_svd(l, step_prec(t - 1), t == 1 ? ows0 : orth_step_set(ows, t - 1), w.sigma,
                          t == 1 ? nullptr : alpha_upd, info, k, t - 1, svd_s);
    if (e == hipSuccess && svd_prev && side != nullptr) e = hipEventRecord(side->svd_done, side->s);
    // Z = X_(k)^T Q3, Y' = X_(k) Z (one pass over X where the fused kernel applies)
    int ns_used = nsplit;
    if (e == hipSuccess)
      e = launch_power_products(tp, v, X, w.qt, l, w.omz, w.part, nsplit, ows.pf_ctr, &nfused, &ns_used, st,
                                info != nullptr ? &info->flags : nullptr);
    // Y = (Y' - alpha Q3) J, then its CholeskyQR. Step 1 needs nothing from
    // the sketch's SVD: alpha_0 = 0, and J_0 only turns the basis inside the
    // span, which leaves the iterate's left singular vectors and values as
    // they are; step 1 factors Y' itself and its own SVD absorbs J_0, except
    // in large modes (rot1), where it waits for J_0 here and applies it.
    if (e == hipSuccess && t > 1 && side != nullptr) e = hipStreamWaitEvent(st, side->svd_done, 0);
    if (e == hipSuccess)
      e = launch_reduce_splits(tp, w.part, ns_used, n * l, ows.Qa, TUCKER_FP64, alpha, w.y64, st);
    if (e == hipSuccess && t == 1 && rot1) e = hipStreamWaitEvent(st, side->log_done, 0);
    if (e == hipSuccess)
      e = launch_orth_qr(n, l, w.y64, t > 1 ? ows.Wm : (rot1 ? ows0.Wm : nullptr), tp, w.qt, orth_step_set(ows, t),
                         cseed, t, st);
  }
  // last small SVD on the caller's stream, after the side SVDs (they share Wm
  // and sigma); then Q = Q3 J (also as Q^T j-major when asked)
  if (e == hipSuccess && q == 1 && side != nullptr && !log_sketch) e = hipStreamWaitEvent(st, side->svd_done, 0);
  if (e == hipSuccess)
    e = launch_orth_svd(l, step_prec(q), q == 0 ? ows0 : orth_step_set(ows, q), w.sigma, q == 0 ? nullptr : alpha_upd,
                        info, k, q, st);
  if (e == hipSuccess) e = launch_orth_rotate(n, l, ows, prec, nullptr, qt_out, w.q64, st);
  // the logging SVD of the sketch joins back before the mode ends (the next
  // mode's sketch reuses its set)
  if (e == hipSuccess && log_sketch) e = hipStreamWaitEvent(st, side->log_done, 0);
  return e == hipSuccess ? TUCKER_OK : dev_check(e, "mode launch");
}

// Algorithm 4 for mode k: the same steps as mode_factor with q_max power
// steps at most; the small SVD of each step evaluates the per-vector-error
// test and the host reads its flag (4 bytes, one stream synchronisation per
// step) before launching the next step. No side stream: the next step's
// launch depends on this step's SVD. *q_used = steps taken.
int mode_factor_pve(const Plan& pl, int k, const void* X, int q_max, double tol, tucker_shift shift, uint64_t seed,
                    tucker_precision prec, tucker_info* info, const SolveWs& w, hipStream_t st, int32_t* q_used) {
  const View3 v = pl.v[k];
  const int l = pl.l[k];
  const int64_t n = v.n, m = pl.m[k];
  const int nsplit = colreduce_splits_for(v, l, prec);
  const OrthWs ows = carve_orth(w.orth, n, l);
  const uint64_t cseed = completion_seed(seed, k);
  double* alpha = w.alpha + k;
  double* alpha_upd = shift == TUCKER_SHIFT_ADAPTIVE ? alpha : nullptr;
  // BF16 operands: FP32 products for the steps that may be the last (as mode_factor's last step)
  const tucker_precision tp = prec == TUCKER_BF16 ? TUCKER_FP32 : prec;
  // FP32 iterates: estimate changes below 1e-6 sigma_t(1) are rounding (the
  // level below which the small SVD already treats directions as noise)
  const SvdPve pve{(int)pl.r[k], tol, tp == TUCKER_FP64 ? 0.0 : 1e-6, alpha, w.sig_hat, w.stop};
  hipError_t e = launch_fill_gaussian(prec == TUCKER_FP64 ? TUCKER_FP64 : TUCKER_FP32, seed, (uint32_t)k, 0, m, l,
                                      true, w.omz, st);
  if (e == hipSuccess)
    e = launch_colreduce(prec, v, X, w.omz, l, w.part, nsplit, st, w.na2 != nullptr ? w.napart : nullptr);
  if (e == hipSuccess && w.na2 != nullptr) e = launch_norm_of_input(prec, v, X, nsplit, w, st);
  if (e == hipSuccess) e = launch_reduce_splits(prec, w.part, nsplit, n * l, nullptr, prec, nullptr, w.y64, st);
  if (e == hipSuccess) e = launch_mode_start(alpha, ows.pf_ctr, st);
  int nfused = 0;  // fused power steps launched since the counter was zeroed
  if (e == hipSuccess) e = launch_orth_qr(n, l, w.y64, nullptr, prec, w.qt, ows, cseed, 0, st);
  if (e == hipSuccess) e = launch_orth_svd(l, prec, ows, w.sigma, nullptr, info, k, 0, st, &pve);
  int t = 0;
  while (e == hipSuccess && t < q_max) {
    ++t;
    // Z = X_(k)^T Q3, Y' = X_(k) Z, Y = (Y' - alpha Q3) J (reading R1), CholeskyQR, small SVD + test
    int ns_used = nsplit;
    e = launch_power_products(tp, v, X, w.qt, l, w.omz, w.part, nsplit, ows.pf_ctr, &nfused, &ns_used, st,
                              info != nullptr ? &info->flags : nullptr);
    if (e == hipSuccess) e = launch_reduce_splits(tp, w.part, ns_used, n * l, ows.Qa, TUCKER_FP64, alpha, w.y64, st);
    if (e == hipSuccess) e = launch_orth_qr(n, l, w.y64, ows.Wm, tp, w.qt, ows, cseed, t, st);
    if (e == hipSuccess) e = launch_orth_svd(l, tp, ows, w.sigma, alpha_upd, info, k, t, st, &pve);
    int halt = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(&halt, w.stop, sizeof(int), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e == hipSuccess && halt) break;
  }
  if (e == hipSuccess) e = launch_orth_rotate(n, l, ows, prec, nullptr, nullptr, w.q64, st);
  *q_used = t;
  return e == hipSuccess ? TUCKER_OK : dev_check(e, "mode launch (per-vector-error)");
}

int solve_holistic(const Plan& pl, const void* A, tucker_shift shift, int32_t q, uint64_t seed,
                   tucker_precision prec, void* G, void* const* U, tucker_info* info, const SolveWs& w, hipStream_t st,
                   int omega_kind);
int solve_modes(const Plan& pl, const void* A, tucker_shift shift, int32_t q, uint64_t seed, tucker_precision prec,
                void* G, void* const* U, tucker_info* info, const SolveWs& w, hipStream_t st, int omega_kind,
                double pve_tol, int32_t* q_used);

int solve(bool st_variant, const tucker_shape* shape, const void* A, const int64_t* ranks, int32_t p, int32_t q,
          tucker_shift shift, uint64_t seed, tucker_precision prec, void* G, void* const* U, tucker_info* info,
          void* ws, size_t ws_bytes, hipStream_t st, double pve_tol = -1.0, int32_t* q_used = nullptr,
          const tucker_options* opt = nullptr, bool one_stream = false) {
  const ProductScope products(opt != nullptr ? opt->fp32_products : TUCKER_FP32_SPLIT);
  Plan pl;
  // with the per-vector-error test q is the largest power count; the plan (and
  // the per-step logs) cover the first TUCKER_MAX_Q steps
  int rc = make_plan(shape, ranks, p, pve_tol >= 0.0 ? std::min<int32_t>(q, TUCKER_MAX_Q) : q, prec, st_variant, &pl,
                     opt);
  if (rc) return rc;
  pl.one_stream = one_stream;
  if (shift != TUCKER_SHIFT_ADAPTIVE && shift != TUCKER_SHIFT_NONE) return fail(TUCKER_EINVAL, "bad shift mode");
  if (A == nullptr || G == nullptr || U == nullptr) return fail(TUCKER_EINVAL, "null tensor, core or factor array");
  for (int k = 0; k < pl.d; ++k)
    if (U[k] == nullptr) return fail(TUCKER_EINVAL, "U[%d] is null", k);
  SolveWs w;
  const size_t need = solve_ws_layout(pl, prec, nullptr, &w);
  if (ws == nullptr || ws_bytes < need)
    return fail(TUCKER_EWORKSPACE, "workspace %zu bytes < required %zu", ws_bytes, need);
  solve_ws_layout(pl, prec, (char*)ws, &w);

  hipError_t e = hipSuccess;
  if (info != nullptr) {
    int32_t ls[TUCKER_MAX_ORDER];
    for (int k = 0; k < pl.d; ++k) ls[k] = pl.l[k];
    e = launch_info_init(info, ls, pl.d, pl.flags, st);
    if (e != hipSuccess) return dev_check(e, "info init");
  }
  const int omega_kind = opt != nullptr ? opt->omega : TUCKER_OMEGA_GAUSSIAN;
  if (pl.holistic) {
    if (pve_tol >= 0.0) return fail(TUCKER_EUNSUPPORTED, "the per-vector-error test runs Algorithm 3 only");
    rc = solve_holistic(pl, A, shift, q, seed, prec, G, U, info, w, st, omega_kind);
    if (rc) return rc;
  } else {
    rc = solve_modes(pl, A, shift, q, seed, prec, G, U, info, w, st, omega_kind, pve_tol, q_used);
    if (rc) return rc;
  }
  if (info != nullptr) {
    int64_t gn = 1;
    for (int k = 0; k < pl.d; ++k) gn *= pl.r[k];
    e = launch_norm2(prec, G, gn, w.normpart, &info->normG2, st);
    if (e == hipSuccess) e = launch_info_rel_error(info, st);
    if (e != hipSuccess) return dev_check(e, "norm launch");
  }
  return TUCKER_OK;
}

// Algorithms 2, 3 and 4 after the plan: every mode's factor, then the core.
int solve_modes(const Plan& pl, const void* A, tucker_shift shift, int32_t q, uint64_t seed, tucker_precision prec,
                void* G, void* const* U, tucker_info* info, const SolveWs& w, hipStream_t st, int omega_kind,
                double pve_tol, int32_t* q_used) {
  const bool st_variant = pl.st;
  hipError_t e = hipSuccess;
  int rc = TUCKER_OK;
  const tucker_precision core_mk = prec == TUCKER_BF16 ? TUCKER_FP32 : prec;
  const void* X = A;
  int64_t cur[TUCKER_MAX_ORDER];
  for (int k = 0; k < pl.d; ++k) cur[k] = pl.dims[k];

  // T-HOSVD: every mode only reads A, so mode 0 runs on the caller's stream
  // and modes 1..d-1 on their own streams (each with its own scratch and SVD
  // side stream), forked from the caller's stream here and joined back before
  // the core chain.
  // Under stream capture the modes run one after another on the caller's
  // stream (each with its side streams, the pattern of the captured ST-HOSVD):
  // the fork of the d - 1 mode streams from one event is not captured.
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  if (!st_variant) {
    const hipError_t ce = hipStreamIsCapturing(st, &cap);
    if (ce != hipSuccess) return dev_check(ce, "hipStreamIsCapturing");
  }
  const bool concurrent =
      !st_variant && pl.d > 1 && pve_tol < 0.0 && !pl.one_stream && cap == hipStreamCaptureStatusNone;
  SideCtx* lanes[TUCKER_MAX_ORDER] = {};
  if (concurrent) {
    for (int k = 1; k < pl.d; ++k) {
      rc = side_ctx(&lanes[k], k);
      if (rc) return rc;
    }
    e = hipEventRecord(lanes[1]->fork, st);
    for (int k = 1; k < pl.d && e == hipSuccess; ++k) e = hipStreamWaitEvent(lanes[k]->ms, lanes[1]->fork, 0);
    if (e != hipSuccess) return dev_check(e, "mode fork");
  }
  bool done[TUCKER_MAX_ORDER] = {};
  for (int i = 0; i < pl.d; ++i) {
    const int k = pl.ord[i];
    const void* Xk = st_variant ? X : A;
    const hipStream_t sk = concurrent && k > 0 ? lanes[k]->ms : st;
    SolveWs wk = w.for_mode(k);
    wk.na2 = (i == 0 && info != nullptr) ? &info->normA2 : nullptr;
    // the tensor mode k works on: A (T-HOSVD), or A with the modes processed
    // before k contracted (ST-HOSVD)
    int64_t curk[TUCKER_MAX_ORDER];
    for (int j = 0; j < pl.d; ++j) curk[j] = (st_variant && done[j]) ? pl.r[j] : pl.dims[j];
    const OmegaSpec om = omega_spec(omega_kind, pl.d, curk, k);
    rc = pve_tol >= 0.0 ? mode_factor_pve(pl, k, Xk, q, pve_tol, shift, seed, prec, info, wk, sk, q_used + k)
                        : mode_factor(pl, k, Xk, q, shift, seed, prec, info, wk, sk, om, concurrent ? k : 0);
    if (rc) return rc;
    e = launch_signfix(prec, wk.q64, pl.v[k].n, pl.l[k], (int)pl.r[k], U[k], wk.ut, sk);
    if (e != hipSuccess) return dev_check(e, "sign rule launch");
    if (st_variant) {
      void* out = (i == pl.d - 1) ? G : w.xbuf[i & 1];
      e = launch_rowcontract(core_mk, pl.v[k], X, wk.ut, 1, pl.v[k].n, (int)pl.r[k], out, false, st);
      if (e != hipSuccess) return dev_check(e, "core launch");
      X = out;
    }
    done[k] = true;
  }
  if (concurrent) {
    for (int k = 1; k < pl.d && e == hipSuccess; ++k) {
      e = hipEventRecord(lanes[k]->join, lanes[k]->ms);
      if (e == hipSuccess) e = hipStreamWaitEvent(st, lanes[k]->join, 0);
    }
    if (e != hipSuccess) return dev_check(e, "mode join");
  }
  if (!st_variant) {
    for (int k = 0; k < pl.d; ++k) {
      const View3 v = view_of(cur, pl.d, k);
      void* out = (k == pl.d - 1) ? G : w.xbuf[k & 1];
      e = launch_rowcontract(core_mk, v, X, U[k], pl.r[k], 1, (int)pl.r[k], out, false, st);
      if (e != hipSuccess) return dev_check(e, "core launch");
      X = out;
      cur[k] = pl.r[k];
    }
  }
  return TUCKER_OK;
}

// The holistic variants (Appendix Algorithms A.2 / B.1 and the T-HOSVD
// analogue). Phase 1: each mode's range finder (mode_factor) keeps all l_k
// columns Q_k, signed by the sign rule; ST contracts B = B x_k Q_k^T at once, T forms B from A after
// the loop. Phase 2: the deterministic (S)T-HOSVD of B (sizes l_k): mode k's
// unfolding (l_k x m) goes to FP64; when m >= l_k its transpose is
// orthonormalised and V_k are the right singular vectors of the R factor,
// else the unfolding itself and V_k are its left singular vectors; then
// U_k = Q_k V_k with the sign rule and the core contraction by the signed V_k.
int solve_holistic(const Plan& pl, const void* A, tucker_shift shift, int32_t q, uint64_t seed,
                   tucker_precision prec, void* G, void* const* U, tucker_info* info, const SolveWs& w, hipStream_t st,
                   int omega_kind) {
  const int d = pl.d;
  const tucker_precision core_mk = prec == TUCKER_BF16 ? TUCKER_FP32 : prec;
  hipError_t e = hipSuccess;
  int rc = TUCKER_OK;
  // phase 1
  const void* X = A;
  bool done[TUCKER_MAX_ORDER] = {};
  for (int i = 0; i < d; ++i) {
    const int k = pl.ord[i];
    int64_t curk[TUCKER_MAX_ORDER];
    for (int j = 0; j < d; ++j) curk[j] = (pl.st && done[j]) ? pl.l[j] : pl.dims[j];
    const OmegaSpec om = omega_spec(omega_kind, d, curk, k);
    SolveWs wk = w;
    wk.q64 = w.hq64[k];
    wk.na2 = (i == 0 && info != nullptr) ? &info->normA2 : nullptr;
    rc = mode_factor(pl, k, pl.st ? X : A, q, shift, seed, prec, info, wk, st, om);
    if (rc) return rc;
    // Q_k with the sign rule (its basis fixes the coordinates the next mode's
    // test matrix multiplies), kept in FP64 and as Q_k^T in the storage precision
    e = launch_signcols(core_mk, w.hq64[k], pl.dims[k], pl.l[k], w.hqt[k], st);
    if (e != hipSuccess) return dev_check(e, "sign rule launch");
    if (pl.st) {
      void* out = (i == d - 1) ? w.bbuf : w.xbuf[i & 1];
      e = launch_rowcontract(core_mk, pl.v[k], X, w.hqt[k], 1, pl.dims[k], pl.l[k], out, false, st);
      if (e != hipSuccess) return dev_check(e, "range contraction launch");
      X = out;
    }
    done[k] = true;
  }
  if (!pl.st) {
    int64_t cur[TUCKER_MAX_ORDER];
    for (int k = 0; k < d; ++k) cur[k] = pl.dims[k];
    X = A;
    for (int k = 0; k < d; ++k) {
      void* out = (k == d - 1) ? w.bbuf : w.xbuf[k & 1];
      e = launch_rowcontract(core_mk, view_of(cur, d, k), X, w.hqt[k], 1, pl.dims[k], pl.l[k], out, false, st);
      if (e != hipSuccess) return dev_check(e, "range contraction launch");
      X = out;
      cur[k] = pl.l[k];
    }
  }
  // phase 2: the deterministic (S)T-HOSVD of B
  int64_t cur[TUCKER_MAX_ORDER];
  for (int k = 0; k < d; ++k) cur[k] = pl.l[k];
  const void* C = w.bbuf;
  for (int i = 0; i < d; ++i) {
    const int k = pl.ord[i];
    const View3 v = view_of(cur, d, k);
    const int64_t lk = pl.l[k];
    const int64_t m = v.P * v.S;
    const bool tall = m >= lk;
    const int64_t rows = tall ? m : lk;
    const int cols = (int)(tall ? lk : m);
    const OrthWs o2 = carve_orth(w.orth2, rows, cols);
    // the unfolding is exact in FP64 whatever the storage: FP64 settings (shifted
    // first CholeskyQR pass, rotations down to l u), so every column of V_k
    // comes out orthonormal, also those at the storage rounding level
    e = launch_unfold64(core_mk, v, pl.st ? C : w.bbuf, tall, w.y2, st);
    if (e == hipSuccess)
      e = launch_orth_qr(rows, cols, w.y2, nullptr, TUCKER_FP64, nullptr, o2,
                         completion_seed(seed, TUCKER_MAX_ORDER + k), 0, st);
    if (e == hipSuccess)
      e = launch_orth_svd(cols, TUCKER_FP64, o2, w.sig2, nullptr, nullptr, -1, -1, st, nullptr,
                          tall ? w.v2 : nullptr);
    if (e == hipSuccess && !tall) e = launch_orth_rotate(rows, cols, o2, core_mk, nullptr, nullptr, w.v2, st);
    if (e == hipSuccess)
      e = launch_assemble(core_mk, w.hq64[k], pl.dims[k], (int)lk, w.v2, cols, (int)pl.r[k], U[k], w.hvt[k], st);
    if (e != hipSuccess) return dev_check(e, "small HOSVD launch");
    if (pl.st) {
      void* out = (i == d - 1) ? G : w.xbuf[i & 1];
      e = launch_rowcontract(core_mk, v, C, w.hvt[k], 1, lk, (int)pl.r[k], out, false, st);
      if (e != hipSuccess) return dev_check(e, "core launch");
      C = out;
      cur[k] = pl.r[k];
    }
  }
  if (!pl.st) {
    X = w.bbuf;
    for (int k = 0; k < d; ++k) {
      void* out = (k == d - 1) ? G : w.xbuf[k & 1];
      e = launch_rowcontract(core_mk, view_of(cur, d, k), X, w.hvt[k], 1, pl.l[k], (int)pl.r[k], out, false, st);
      if (e != hipSuccess) return dev_check(e, "core launch");
      X = out;
      cur[k] = pl.r[k];
    }
  }
  return TUCKER_OK;
}

int check_op(const tucker_shape* shape, int32_t mode, int64_t l, tucker_precision prec, View3* v, int64_t* m) {
  int64_t numel;
  int rc = check_shape(shape, &numel);
  if (rc) return rc;
  if (!valid_prec(prec)) return fail(TUCKER_EINVAL, "bad precision %d", (int)prec);
  if (mode < 0 || mode >= shape->order) return fail(TUCKER_EINVAL, "mode %d outside 0..%d", mode, shape->order - 1);
  *v = view_of(shape->dims, shape->order, mode);
  *m = numel / v->n;
  if (l < 1 || l > TUCKER_MAX_L || l > v->n || l > *m)
    return fail(TUCKER_EINVAL, "l = %lld outside 1..min(%d, n = %lld, m = %lld)", (long long)l, TUCKER_MAX_L,
                (long long)v->n, (long long)*m);
  return TUCKER_OK;
}

struct OpWs {
  void* omz;
  void* part;
  double* y64;
  void* orth;
  void* qt;  // Q^T (l x n, storage precision): the j-major operand the solve's products read
};

size_t op_ws_layout(const View3& v, int64_t m, int l, tucker_precision prec, char* base, OpWs* w) {
  size_t off = 0;
  auto take = [&](size_t bytes) -> void* {
    void* p = base ? base + off : nullptr;
    off += align_up(bytes);
    return p;
  };
  w->omz = take((size_t)m * l * elem_bytes(prec));
  w->part = take(colreduce_part_bytes(v, l, prec));
  w->y64 = (double*)take((size_t)v.n * l * 8);
  w->orth = take(orth_ws_bytes(v.n, l));
  w->qt = take((size_t)v.n * l * elem_bytes(prec));
  return off;
}


// ---- batched solves --------------------------------------------------------
constexpr uint32_t kBatchMagic = 0x54424154u;  // plan header tag

struct BatchHeader {
  uint32_t magic;
  int32_t capacity, order, q, lclass, nphases;
  size_t table_bytes;
  char* ws;
};
struct PhaseRec {
  int32_t kind;
  int32_t pad;
  size_t hdr_off, desc_off;  // within the table image
  double bytes, flops;       // algorithmic traffic and work of the phase (launch timing)
};

// The fixed phase sequence for (order, q).
std::vector<BatchKind> batch_phases(int d, int q) {
  std::vector<BatchKind> ph{BK_INIT};
  const BatchKind orth[] = {BK_GRAM, BK_PASS, BK_PASS, BK_PASS, BK_SVD};
  for (int k = 0; k < d; ++k) {
    for (BatchKind b : {BK_FILL, BK_CR_SPLIT, BK_CR_COLS, BK_REDUCE}) ph.push_back(b);
    for (BatchKind b : orth) ph.push_back(b);
    for (int t = 1; t <= q; ++t) {
      for (BatchKind b : {BK_RC_SPLIT, BK_RC_COLS, BK_CR_SPLIT, BK_CR_COLS, BK_REDUCE}) ph.push_back(b);
      for (BatchKind b : orth) ph.push_back(b);
    }
    for (BatchKind b : {BK_ROTATE, BK_SIGNFIX, BK_RC_SPLIT, BK_RC_COLS}) ph.push_back(b);
  }
  return ph;
}

size_t batch_table_layout(int cap, int d, int q, std::vector<PhaseRec>* recs) {
  const std::vector<BatchKind> ph = batch_phases(d, q);
  size_t off = 0;
  if (recs) recs->clear();
  for (BatchKind k : ph) {
    PhaseRec r;
    r.kind = (int32_t)k;
    r.pad = 0;
    r.bytes = r.flops = 0.0;
    r.hdr_off = off;
    off += align_up((size_t)(cap + 10) * sizeof(int));  // item table and the 8 claim counters
    r.desc_off = off;
    off += align_up((size_t)cap * batch_desc_bytes(k));
    if (recs) recs->push_back(r);
  }
  return off;
}

size_t batch_plan_bytes(int cap, int d, int q) {
  return align_up(sizeof(BatchHeader)) + align_up(batch_phases(d, q).size() * sizeof(PhaseRec)) +
         batch_table_layout(cap, d, q, nullptr);
}

int batch_item_plan(const tucker_batch_item* it, int32_t p, int32_t q, Plan* pl) {
  if (it == nullptr) return fail(TUCKER_EINVAL, "null item");
  int rc = make_plan(&it->shape, it->ranks, p, q, TUCKER_FP32, true, pl);
  if (rc) return rc;
  if (it->A == nullptr || it->G == nullptr) return fail(TUCKER_EINVAL, "item with null tensor or core");
  for (int k = 0; k < pl->d; ++k)
    if (it->U[k] == nullptr) return fail(TUCKER_EINVAL, "item with null U[%d]", k);
  return TUCKER_OK;
}

// Algorithmic HBM bytes and flops of one item's mode product in a phase (the
// unfolding read once, the small operand read once; FP32 storage).
void batch_phase_work(BatchKind kind, int k, int role, const Plan& pl, double* bytes, double* flops) {
  const View3 v = pl.v[k];
  const double N = (double)v.P * v.n * v.S, m = (double)pl.m[k];
  const bool cr = (kind == BK_CR_SPLIT && v.S > 1) || (kind == BK_CR_COLS && v.S == 1);
  const bool rc = (kind == BK_RC_SPLIT && v.S > 1) || (kind == BK_RC_COLS && v.S == 1);
  if (!cr && !rc) return;
  const double w = rc && role == 1 ? (double)pl.r[k] : (double)pl.l[k];
  *bytes += 4.0 * (N + m * w);
  *flops += 2.0 * N * w;
}

// Splits of a request's column reduction inside a batch: the batch already
// fills the device, so a split covers at least 2048 columns (S > 1) or 8 steps
// (S == 1). A small unfolding (fewer than 8 such splits) takes up to 8 splits of
// at least 16 stages of 32 columns, as long as the partials (n x l per split)
// stay within 1/16 of the unfolding's bytes: its few long items would
// otherwise end the launch. Never more splits than the request's own workspace
// holds. Depends on the request's shape only, so a request computes the same
// alone and in any mix.
int batch_colreduce_splits(const View3& v, int l) {
  int64_t nsteps, spp;
  int nrb;
  cr_geometry(v, &nsteps, &spp, &nrb);
  int64_t ns = std::max<int64_t>(1, nsteps / (v.S > 1 ? 32 : 8));
  if (v.S > 1 && ns < 8) {
    int64_t ns32, spp32;
    cr_split_geometry(v, &ns32, &spp32, &nrb);
    ns = std::max<int64_t>(ns, std::min<int64_t>({8, ns32 / 16, v.P * v.S / (16 * (int64_t)l)}));
  }
  ns = std::min<int64_t>(ns, colreduce_splits(v, l));
  // a multiple of 8 from 8 up: the row blocks of one split then share an XCD
  // (and its L2 copy of the split's slice of the skinny operand)
  return (int)(ns >= 8 ? ns / 8 * 8 : ns);
}

// Fills one phase's descriptor for item b (returns its work items).
int64_t batch_desc(BatchKind kind, int k, int t, int role, const Plan& pl, const SolveWs& w,
                   const tucker_batch_item& it, tucker_shift shift, int d, int q, void* dst) {
  const View3 v = pl.v[k];
  const int l = pl.l[k], r = (int)pl.r[k];
  const int64_t n = v.n, m = pl.m[k];
  const OrthWs ows = carve_orth(w.orth, n, l);
  const void* X = k == 0 ? it.A : w.xbuf[(k - 1) & 1];
  const int nsplit = batch_colreduce_splits(v, l);
  const int nblk = (int)((n + 63) / 64);
  double* alpha = w.alpha + k;
  switch (kind) {
    case BK_INIT: {
      BInit* b = (BInit*)dst;
      b->info = it.info;
      b->alpha = w.alpha;
      for (int j = 0; j < TUCKER_MAX_ORDER; ++j) b->l[j] = j < d ? pl.l[j] : 0;
      b->d = d;
      b->flags = pl.flags;
      return 1;
    }
    case BK_FILL: {
      BFill* b = (BFill*)dst;
      b->out = (float*)w.omz;
      b->seed = it.seed;
      b->rows = m;
      b->ld = m;
      b->mode = (uint32_t)k;
      b->cols = l;
      return (m * ((l + 3) / 4) + 255) / 256;
    }
    case BK_CR_SPLIT:
    case BK_CR_COLS: {
      int64_t nsteps, spp;
      int nrb;
      if (kind == BK_CR_SPLIT)
        cr_split_geometry(v, &nsteps, &spp, &nrb);
      else
        cr_geometry(v, &nsteps, &spp, &nrb);
      if (kind == BK_CR_SPLIT) {
        BCrSplit* b = (BCrSplit*)dst;
        b->X = (const float*)X;
        b->Bt = (const float*)w.omz;
        b->part = (float*)w.part;
        b->n = n;
        b->S = v.S;
        b->m = m;
        b->spp = spp;
        b->nsteps = nsteps;
        b->l = l;
        b->nsplit = nsplit;
        b->nrb = nrb;
        return v.S > 1 ? cr_split_items(n, nsplit) : 0;
      }
      BCrCols* b = (BCrCols*)dst;
      b->X = (const float*)X;
      b->Bt = (const float*)w.omz;
      b->part = (float*)w.part;
      b->P = v.P;
      b->n = n;
      b->nsteps = nsteps;
      b->l = l;
      b->nsplit = nsplit;
      b->nrb = nrb;
      return v.S == 1 ? cr_cols_items(n, nsplit) : 0;
    }
    case BK_REDUCE: {
      BReduce* b = (BReduce*)dst;
      b->part = (const float*)w.part;
      b->qsub = t == 0 ? nullptr : ows.Qa;
      b->alpha = alpha;
      b->Y = w.y64;
      b->nl = n * l;
      b->nsplit = nsplit;
      return (n * l + 31) / 32;
    }
    case BK_RC_SPLIT:
    case BK_RC_COLS: {
      // power step (role 0): Z = X_(k)^T Q3, j-major; core (role 1): X x_k U_k^T
      const bool core = role == 1;
      const int lw = core ? r : l;
      const void* W = core ? w.ut : w.qt;
      void* out = core ? (k == d - 1 ? it.G : w.xbuf[k & 1]) : w.omz;
      if (kind == BK_RC_SPLIT) {
        BRcSplit* b = (BRcSplit*)dst;
        int64_t tpp;
        const int64_t ntiles = rc_split_tiles(v, &tpp);  // each wave owns a tile and all n rows
        b->X = (const float*)X;
        b->W = (const float*)W;
        b->out = (float*)out;
        b->n = n;
        b->S = v.S;
        b->wsi = 1;
        b->wsj = n;
        b->tpp = tpp;
        b->ntiles = ntiles;
        b->osp = core ? (int64_t)lw * v.S : v.S;
        b->osj = core ? v.S : m;
        b->lw = lw;
        return v.S > 1 ? (ntiles + 3) / 4 : 0;
      }
      BRcCols* b = (BRcCols*)dst;
      b->X = (const float*)X;
      b->W = (const float*)W;
      b->out = (float*)out;
      b->P = v.P;
      b->n = n;
      b->wsi = 1;
      b->wsj = n;
      b->osp = core ? lw : 1;
      b->osj = core ? 1 : m;
      b->lw = lw;
      return v.S == 1 ? (v.P + 63) / 64 : 0;
    }
    case BK_GRAM: {
      BGram* b = (BGram*)dst;
      b->Y = w.y64;
      b->Wm = t <= 1 ? nullptr : ows.Wm;  // as the one-request path: step 1 factors the unrotated iterate
      b->part = ows.part;
      b->status = ows.status;
      b->n = n;
      b->l = l;
      return nblk;
    }
    case BK_PASS: {
      BPass* b = (BPass*)dst;
      const size_t pstride = align_up((size_t)nblk * l * l * sizeof(double)) / sizeof(double);
      double* p0 = ows.part;
      double* p1 = ows.part + pstride;
      const uint32_t tag = 0x100u + 16u * (uint32_t)t;
      b->Qin = role == 0 ? w.y64 : ows.Qa;
      b->part_in = role == 1 ? p1 : p0;
      b->Qout = ows.Qa;
      b->qt = w.qt;
      b->part_out = role == 0 ? p1 : (role == 1 ? p0 : nullptr);
      b->Rg = ows.R + (size_t)role * TUCKER_MAX_L * TUCKER_MAX_L;
      b->defic = ows.defic + role * TUCKER_MAX_L;
      b->status = ows.status;
      b->cseed = completion_seed(it.seed, k);
      b->tau = role == 0 ? 1e-12 : std::max(1e-14, 4.0 * (double)n * 2.220446049250313e-16);
      b->shift_scale = 0.0;
      b->eps3 = 1e-10;
      b->n = n;
      b->l = l;
      b->nblk = nblk;
      b->role = role;
      b->ctag = tag + 1 + (uint32_t)role;
      return nblk;
    }
    case BK_SVD: {
      // with power steps to follow, the sketch's SVD feeds nothing (alpha_0 = 0
      // and step 1 factors the unrotated iterate): it only logs, so it runs for
      // the items that keep a log
      if (t == 0 && q > 0 && it.info == nullptr) return 0;
      BSvd* b = (BSvd*)dst;
      b->Rg = ows.R;
      b->status = ows.status;
      b->Wm = ows.Wm;
      b->sigma = w.sigma;
      b->alpha = (t == 0 || shift != TUCKER_SHIFT_ADAPTIVE) ? nullptr : alpha;
      b->info = it.info;
      b->tol = 1e-8;
      b->negl = 1e-6;
      b->l = l;
      b->mode = k;
      b->step = t;
      return 1;
    }
    case BK_ROTATE: {
      BRotate* b = (BRotate*)dst;
      b->Q3 = ows.Qa;
      b->Wm = ows.Wm;
      b->q64 = w.q64;
      b->n = n;
      b->l = l;
      return (n * l + 255) / 256;
    }
    case BK_SIGNFIX: {
      BSignfix* b = (BSignfix*)dst;
      b->Q = w.q64;
      b->U = (float*)it.U[k];
      b->Ut = (float*)w.ut;
      b->n = n;
      b->l = l;
      b->r = r;
      return r;
    }
    default:
      return 0;
  }
}

}  // namespace

extern "C" {

const char* tucker_status_string(int status) {
  if (status != 0 && status == g_err_code && !g_err_text.empty()) return g_err_text.c_str();
  switch (status) {
    case TUCKER_OK: return "ok";
    case TUCKER_EINVAL: return "invalid argument";
    case TUCKER_EWORKSPACE: return "workspace too small";
    case TUCKER_EDEVICE: return "device error";
    case TUCKER_EUNSUPPORTED: return "unsupported by the library";
  }
  return "unknown status";
}

size_t tucker_workspace_bytes(const tucker_shape* shape, const int64_t* ranks, int32_t p, int32_t q,
                              tucker_precision prec, int32_t sequential) {
  Plan pl;
  if (make_plan(shape, ranks, p, q, prec, sequential != 0, &pl)) return 0;
  SolveWs w;
  return solve_ws_layout(pl, prec, nullptr, &w);
}

size_t tucker_op_workspace_bytes(const tucker_shape* shape, int32_t mode, int64_t l, tucker_precision prec) {
  View3 v;
  int64_t m;
  if (check_op(shape, mode, l, prec, &v, &m)) return 0;
  OpWs w;
  return op_ws_layout(v, m, (int)l, prec, nullptr, &w);
}

int tucker_fill_gaussian(uint64_t seed, int32_t mode, int64_t row0, int64_t rows, int64_t cols,
                         tucker_precision prec, void* out, hipStream_t stream) {
  if (!valid_prec(prec)) return fail(TUCKER_EINVAL, "bad precision %d", (int)prec);
  if (rows < 0 || cols < 0 || row0 < 0) return fail(TUCKER_EINVAL, "negative rows, cols or row0");
  if (mode < 0 || mode >= TUCKER_MAX_ORDER) return fail(TUCKER_EINVAL, "mode %d outside 0..7", mode);
  if (cols > ((int64_t)1 << 30) || rows > ((int64_t)1 << 40)) return fail(TUCKER_EINVAL, "matrix too large");
  if (rows * cols == 0) return TUCKER_OK;
  if (out == nullptr) return fail(TUCKER_EINVAL, "out is null");
  return dev_check(launch_fill_gaussian(prec == TUCKER_FP64 ? TUCKER_FP64 : TUCKER_FP32, seed, (uint32_t)mode, row0,
                                        rows, (int)cols, false, out, stream),
                   "fill launch");
}

int tucker_sketch(const tucker_shape* shape, int32_t mode, const void* X, int64_t l, uint64_t seed,
                  tucker_precision prec, void* Y, void* ws, size_t ws_bytes, hipStream_t stream) {
  View3 v;
  int64_t m;
  int rc = check_op(shape, mode, l, prec, &v, &m);
  if (rc) return rc;
  if (X == nullptr || Y == nullptr) return fail(TUCKER_EINVAL, "null X or Y");
  OpWs w;
  const size_t need = op_ws_layout(v, m, (int)l, prec, nullptr, &w);
  if (ws == nullptr || ws_bytes < need) return fail(TUCKER_EWORKSPACE, "workspace %zu < %zu", ws_bytes, need);
  op_ws_layout(v, m, (int)l, prec, (char*)ws, &w);
  const int nsplit = colreduce_splits_for(v, (int)l, prec);
  hipError_t e = launch_fill_gaussian(prec == TUCKER_FP64 ? TUCKER_FP64 : TUCKER_FP32, seed, (uint32_t)mode, 0, m,
                                      (int)l, true, w.omz, stream);
  if (e == hipSuccess) e = launch_colreduce(prec, v, X, w.omz, (int)l, w.part, nsplit, stream);
  // the fixed-order sum is FP64; FP32 and BF16 calls store it in FP32
  double* y64 = prec == TUCKER_FP64 ? (double*)Y : w.y64;
  if (e == hipSuccess) e = launch_reduce_splits(prec, w.part, nsplit, v.n * l, nullptr, prec, nullptr, y64, stream);
  if (e == hipSuccess && prec != TUCKER_FP64) e = launch_convert_from_f64(TUCKER_FP32, y64, v.n * l, Y, stream);
  return dev_check(e, "sketch launch");
}

int tucker_shifted_power(const tucker_shape* shape, int32_t mode, const void* X, int64_t l, const void* Q,
                         double* alpha, int32_t flags, tucker_precision prec, void* out, double* sigma, void* ws,
                         size_t ws_bytes, hipStream_t stream) {
  View3 v;
  int64_t m;
  int rc = check_op(shape, mode, l, prec, &v, &m);
  if (rc) return rc;
  const bool raw = (flags & TUCKER_POWER_RAW) != 0;
  if (X == nullptr || Q == nullptr || alpha == nullptr || out == nullptr || (!raw && sigma == nullptr))
    return fail(TUCKER_EINVAL, "null argument");
  if (out == Q) return fail(TUCKER_EINVAL, "out aliases Q");
  OpWs w;
  const size_t need = op_ws_layout(v, m, (int)l, prec, nullptr, &w);
  if (ws == nullptr || ws_bytes < need) return fail(TUCKER_EWORKSPACE, "workspace %zu < %zu", ws_bytes, need);
  op_ws_layout(v, m, (int)l, prec, (char*)ws, &w);
  const int nsplit = colreduce_splits_for(v, (int)l, prec);
  double* y = raw ? (double*)out : w.y64;
  hipError_t e;
  int ns_used = nsplit;
  if (power_fused_launch_splits(v, (int)l, prec) > 0 && v.n <= m) {
    // the fused pass reads Q j-major: transposed into the space of Z, which it does not use
    const OrthWs ows = carve_orth(w.orth, v.n, (int)l);
    e = launch_transpose_f32((const float*)Q, v.n, (int)l, (float*)w.omz, stream);
    if (e == hipSuccess) e = launch_mode_start(nullptr, ows.pf_ctr, stream);
    int nfused = 0;
    if (e == hipSuccess)
      e = launch_power_products(prec, v, X, w.omz, (int)l, nullptr, w.part, nsplit, ows.pf_ctr, &nfused, &ns_used,
                                stream);
  } else if (prec != TUCKER_FP64) {
    // Q^T j-major, as the solve's power steps read it (the same kernels run)
    e = launch_transpose_f32((const float*)Q, v.n, (int)l, (float*)w.qt, stream);
    if (e == hipSuccess) e = launch_rowcontract(prec, v, X, w.qt, 1, v.n, (int)l, w.omz, true, stream);
    if (e == hipSuccess) e = launch_colreduce(prec, v, X, w.omz, (int)l, w.part, nsplit, stream);
  } else {
    e = launch_rowcontract(prec, v, X, Q, l, 1, (int)l, w.omz, true, stream);
    if (e == hipSuccess) e = launch_colreduce(prec, v, X, w.omz, (int)l, w.part, nsplit, stream);
  }
  if (e == hipSuccess)
    e = launch_reduce_splits(prec, w.part, ns_used, v.n * l, Q, prec == TUCKER_FP64 ? TUCKER_FP64 : TUCKER_FP32,
                             alpha, y, stream);
  if (e == hipSuccess && !raw) {
    const OrthWs ows = carve_orth(w.orth, v.n, (int)l);
    e = launch_orth(v.n, (int)l, y, prec, out, nullptr, nullptr, sigma, alpha, nullptr, -1, -1, ows,
                    completion_seed(0x5eedull, mode), stream);
  }
  return dev_check(e, "power step launch");
}

int tucker_orth(int64_t n, int64_t l, const double* Y, tucker_precision prec, void* Q, double* sigma, void* ws,
                size_t ws_bytes, hipStream_t stream) {
  if (!valid_prec(prec)) return fail(TUCKER_EINVAL, "bad precision %d", (int)prec);
  if (l < 1 || l > TUCKER_MAX_L || n < l) return fail(TUCKER_EINVAL, "need 1 <= l <= min(n, %d)", TUCKER_MAX_L);
  if (Y == nullptr || Q == nullptr || sigma == nullptr) return fail(TUCKER_EINVAL, "null argument");
  const size_t need = orth_ws_bytes(n, (int)l);
  if (ws == nullptr || ws_bytes < need) return fail(TUCKER_EWORKSPACE, "workspace %zu < %zu", ws_bytes, need);
  const OrthWs ows = carve_orth(ws, n, (int)l);
  return dev_check(launch_orth(n, (int)l, const_cast<double*>(Y), prec, Q, nullptr, nullptr, sigma, nullptr, nullptr, -1, -1, ows,
                               completion_seed(0x0a7bull, 0), stream),
                   "orth launch");
}

int tucker_core(const tucker_shape* shape, int32_t mode, const void* X, const void* U, int64_t r,
                tucker_precision prec, void* Xout, hipStream_t stream) {
  int64_t numel;
  int rc = check_shape(shape, &numel);
  if (rc) return rc;
  if (!valid_prec(prec)) return fail(TUCKER_EINVAL, "bad precision %d", (int)prec);
  if (mode < 0 || mode >= shape->order) return fail(TUCKER_EINVAL, "mode %d outside 0..%d", mode, shape->order - 1);
  if (r < 1 || r > TUCKER_MAX_L) return fail(TUCKER_EINVAL, "r = %lld outside 1..%d", (long long)r, TUCKER_MAX_L);
  if (X == nullptr || U == nullptr || Xout == nullptr) return fail(TUCKER_EINVAL, "null argument");
  const View3 v = view_of(shape->dims, shape->order, mode);
  return dev_check(launch_rowcontract(prec == TUCKER_BF16 ? TUCKER_FP32 : prec, v, X, U, r, 1, (int)r, Xout, false,
                                      stream),
                   "core launch");
}

int tucker_norm2(const void* X, int64_t numel, tucker_precision prec, double* out, void* ws, size_t ws_bytes,
                 hipStream_t stream) {
  if (!valid_prec(prec)) return fail(TUCKER_EINVAL, "bad precision %d", (int)prec);
  if (numel < 0 || X == nullptr || out == nullptr) return fail(TUCKER_EINVAL, "null argument or negative size");
  if (ws == nullptr || ws_bytes < TUCKER_NORM2_WS_BYTES)
    return fail(TUCKER_EWORKSPACE, "workspace %zu < %d", ws_bytes, TUCKER_NORM2_WS_BYTES);
  return dev_check(launch_norm2(prec, X, numel, (double*)ws, out, stream), "norm launch");
}

int tucker_rthosvd(const tucker_shape* shape, const void* A, const int64_t* ranks, int32_t p, int32_t q,
                   tucker_shift shift, uint64_t seed, tucker_precision prec, void* G, void* const* U, tucker_info* info,
                   void* ws, size_t ws_bytes, hipStream_t stream) {
  return solve(false, shape, A, ranks, p, q, shift, seed, prec, G, U, info, ws, ws_bytes, stream);
}

int tucker_rsthosvd(const tucker_shape* shape, const void* A, const int64_t* ranks, int32_t p, int32_t q,
                    tucker_shift shift, uint64_t seed, tucker_precision prec, void* G, void* const* U,
                    tucker_info* info, void* ws, size_t ws_bytes, hipStream_t stream) {
  return solve(true, shape, A, ranks, p, q, shift, seed, prec, G, U, info, ws, ws_bytes, stream);
}

int tucker_rsthosvd_noalloc(const tucker_shape* shape, const void* A, const int64_t* ranks, int32_t p, int32_t q,
                            tucker_shift shift, uint64_t seed, tucker_precision prec, void* G, void* const* U,
                            tucker_info* info, hipStream_t stream) {
  Plan pl;
  int rc = make_plan(shape, ranks, p, q, prec, true, &pl);
  if (rc) return rc;
  SolveWs w;
  const size_t need = solve_ws_layout(pl, prec, nullptr, &w);
  if (need > TUCKER_NOALLOC_SCRATCH_BYTES)
    return fail(TUCKER_EWORKSPACE, "this solve needs %zu bytes of scratch; the static scratch holds %zu", need,
                (size_t)TUCKER_NOALLOC_SCRATCH_BYTES);
  void* ws = nullptr;
  rc = noalloc_scratch(&ws);
  if (rc) return rc;
  return solve(true, shape, A, ranks, p, q, shift, seed, prec, G, U, info, ws, TUCKER_NOALLOC_SCRATCH_BYTES, stream,
               -1.0, nullptr, nullptr, /*one_stream=*/true);
}

// Field checks of an options struct (the order itself is checked against
// the tensor order by make_plan).
static int check_options(const tucker_options* opt) {
  if (opt == nullptr) return TUCKER_OK;
  if (opt->omega < TUCKER_OMEGA_GAUSSIAN || opt->omega > TUCKER_OMEGA_KR_UNIFORM)
    return fail(TUCKER_EINVAL, "unknown test-matrix kind %d", opt->omega);
  if (opt->order_kind < TUCKER_ORDER_NATURAL || opt->order_kind > TUCKER_ORDER_DECREASING)
    return fail(TUCKER_EINVAL, "unknown order kind %d", opt->order_kind);
  if (opt->holistic != 0 && opt->holistic != 1) return fail(TUCKER_EINVAL, "holistic = %d is not 0 or 1", opt->holistic);
  if (opt->fp32_products != TUCKER_FP32_SPLIT && opt->fp32_products != TUCKER_FP32_NATIVE)
    return fail(TUCKER_EINVAL, "fp32_products = %d is not 0 or 1", opt->fp32_products);
  for (int i = 0; i < 4; ++i)
    if (opt->reserved[i] != 0) return fail(TUCKER_EINVAL, "tucker_options.reserved[%d] is not zero", i);
  return TUCKER_OK;
}

size_t tucker_workspace_bytes_ex(const tucker_shape* shape, const int64_t* ranks, int32_t p, int32_t q,
                                 tucker_precision prec, int32_t sequential, const tucker_options* opt) {
  if (check_options(opt)) return 0;
  Plan pl;
  if (make_plan(shape, ranks, p, q, prec, sequential != 0, &pl, opt)) return 0;
  SolveWs w;
  return solve_ws_layout(pl, prec, nullptr, &w);
}

int tucker_rthosvd_ex(const tucker_shape* shape, const void* A, const int64_t* ranks, int32_t p, int32_t q,
                      tucker_shift shift, uint64_t seed, tucker_precision prec, const tucker_options* opt, void* G,
                      void* const* U, tucker_info* info, void* ws, size_t ws_bytes, hipStream_t stream) {
  const int rc = check_options(opt);
  if (rc) return rc;
  return solve(false, shape, A, ranks, p, q, shift, seed, prec, G, U, info, ws, ws_bytes, stream, -1.0, nullptr, opt);
}

int tucker_rsthosvd_ex(const tucker_shape* shape, const void* A, const int64_t* ranks, int32_t p, int32_t q,
                       tucker_shift shift, uint64_t seed, tucker_precision prec, const tucker_options* opt, void* G,
                       void* const* U, tucker_info* info, void* ws, size_t ws_bytes, hipStream_t stream) {
  const int rc = check_options(opt);
  if (rc) return rc;
  return solve(true, shape, A, ranks, p, q, shift, seed, prec, G, U, info, ws, ws_bytes, stream, -1.0, nullptr, opt);
}

int tucker_fill_test_matrix(int32_t kind, uint64_t seed, int32_t mode, int32_t d, const int64_t* dims, int64_t row0,
                            int64_t rows, int64_t cols, tucker_precision prec, void* out, hipStream_t stream) {
  if (!valid_prec(prec)) return fail(TUCKER_EINVAL, "bad precision %d", (int)prec);
  if (kind < TUCKER_OMEGA_GAUSSIAN || kind > TUCKER_OMEGA_KR_UNIFORM)
    return fail(TUCKER_EINVAL, "unknown test-matrix kind %d", kind);
  if (d < 1 || d > TUCKER_MAX_ORDER) return fail(TUCKER_EINVAL, "order %d outside 1..%d", d, TUCKER_MAX_ORDER);
  if (mode < 0 || mode >= d) return fail(TUCKER_EINVAL, "mode %d outside 0..%d", mode, d - 1);
  if (dims == nullptr) return fail(TUCKER_EINVAL, "dims is null");
  for (int i = 0; i < d; ++i)
    if (dims[i] < 1) return fail(TUCKER_EINVAL, "dims[%d] = %lld < 1", i, (long long)dims[i]);
  if (rows < 0 || cols < 0 || row0 < 0) return fail(TUCKER_EINVAL, "negative rows, cols or row0");
  if (cols > ((int64_t)1 << 30) || rows > ((int64_t)1 << 40)) return fail(TUCKER_EINVAL, "matrix too large");
  if (rows * cols == 0) return TUCKER_OK;
  if (out == nullptr) return fail(TUCKER_EINVAL, "out is null");
  const OmegaSpec sp = omega_spec(kind, d, dims, mode);
  return dev_check(launch_fill_omega(sp, prec == TUCKER_FP64 ? TUCKER_FP64 : TUCKER_FP32, seed, (uint32_t)mode, row0,
                                     rows, (int)cols, false, out, stream),
                   "fill launch");
}

int tucker_rsthosvd_pve(const tucker_shape* shape, const void* A, const int64_t* ranks, int32_t p, int32_t q_max,
                        double tol, tucker_shift shift, uint64_t seed, tucker_precision prec, void* G, void* const* U,
                        tucker_info* info, int32_t* q_used, void* ws, size_t ws_bytes, hipStream_t stream) {
  if (q_max < 1 || q_max > TUCKER_MAX_Q_PVE)
    return fail(TUCKER_EINVAL, "q_max = %d outside 1..%d", q_max, TUCKER_MAX_Q_PVE);
  if (!(tol >= 0.0)) return fail(TUCKER_EINVAL, "tol must be >= 0 (got %g)", tol);
  if (q_used == nullptr) return fail(TUCKER_EINVAL, "q_used is null");
  return solve(true, shape, A, ranks, p, q_max, shift, seed, prec, G, U, info, ws, ws_bytes, stream, tol, q_used);
}

int tucker_rthosvd_pve(const tucker_shape* shape, const void* A, const int64_t* ranks, int32_t p, int32_t q_max,
                       double tol, tucker_shift shift, uint64_t seed, tucker_precision prec, void* G, void* const* U,
                       tucker_info* info, int32_t* q_used, void* ws, size_t ws_bytes, hipStream_t stream) {
  if (q_max < 1 || q_max > TUCKER_MAX_Q_PVE)
    return fail(TUCKER_EINVAL, "q_max = %d outside 1..%d", q_max, TUCKER_MAX_Q_PVE);
  if (!(tol >= 0.0)) return fail(TUCKER_EINVAL, "tol must be >= 0 (got %g)", tol);
  if (q_used == nullptr) return fail(TUCKER_EINVAL, "q_used is null");
  return solve(false, shape, A, ranks, p, q_max, shift, seed, prec, G, U, info, ws, ws_bytes, stream, tol, q_used);
}

size_t tucker_batch_plan_bytes(int32_t capacity, int32_t order, int32_t q) {
  if (capacity < 1 || capacity > 4096 || order < 1 || order > TUCKER_MAX_ORDER || q < 0 || q > TUCKER_MAX_Q) return 0;
  return batch_plan_bytes(capacity, order, q);
}

size_t tucker_batch_table_bytes(int32_t capacity, int32_t order, int32_t q) {
  if (capacity < 1 || capacity > 4096 || order < 1 || order > TUCKER_MAX_ORDER || q < 0 || q > TUCKER_MAX_Q) return 0;
  return align_up(batch_table_layout(capacity, order, q, nullptr));
}

size_t tucker_batch_item_bytes(const tucker_batch_item* item, int32_t p, int32_t q) {
  Plan pl;
  if (batch_item_plan(item, p, q, &pl)) return 0;
  SolveWs w;
  return align_up(solve_ws_layout(pl, TUCKER_FP32, nullptr, &w));
}

int tucker_batch_plan(int32_t capacity, int32_t order, int32_t lclass, int32_t nitems, const tucker_batch_item* items,
                      int32_t p, int32_t q, tucker_shift shift, void* ws, size_t ws_bytes, void* plan,
                      size_t plan_bytes) {
  if (capacity < 1 || capacity > 4096) return fail(TUCKER_EINVAL, "capacity %d outside 1..4096", capacity);
  if (lclass != 16 && lclass != 32 && lclass != 48 && lclass != 64)
    return fail(TUCKER_EINVAL, "lclass %d is not 16, 32, 48 or 64", lclass);
  if (nitems < 0 || nitems > capacity) return fail(TUCKER_EINVAL, "nitems %d outside 0..capacity", nitems);
  if (nitems > 0 && items == nullptr) return fail(TUCKER_EINVAL, "items is null");
  if (shift != TUCKER_SHIFT_ADAPTIVE && shift != TUCKER_SHIFT_NONE) return fail(TUCKER_EINVAL, "bad shift mode");
  if (q < 0 || q > TUCKER_MAX_Q) return fail(TUCKER_EINVAL, "power count q = %d outside 0..%d", q, TUCKER_MAX_Q);
  if (ws == nullptr || plan == nullptr) return fail(TUCKER_EINVAL, "null workspace or plan");
  const int d = order;
  if (d < 1 || d > TUCKER_MAX_ORDER) return fail(TUCKER_EINVAL, "order %d outside 1..%d", d, TUCKER_MAX_ORDER);
  const size_t need_plan = batch_plan_bytes(capacity, d, q);
  if (plan_bytes < need_plan) return fail(TUCKER_EWORKSPACE, "plan buffer %zu < %zu", plan_bytes, need_plan);
  std::vector<PhaseRec> recs;
  const size_t tb = batch_table_layout(capacity, d, q, &recs);
  // per item plans and workspace carve
  std::vector<Plan> pls((size_t)nitems);
  std::vector<SolveWs> wss((size_t)nitems);
  size_t off = align_up(tb);
  for (int b = 0; b < nitems; ++b) {
    if (items[b].shape.order != d) return fail(TUCKER_EINVAL, "item %d has order %d, batch order %d", b,
                                               items[b].shape.order, d);
    int rc = batch_item_plan(&items[b], p, q, &pls[b]);
    if (rc) return rc;
    for (int k = 0; k < d; ++k)
      if (pls[b].l[k] > lclass)
        return fail(TUCKER_EUNSUPPORTED, "item %d: l[%d] = %d exceeds lclass %d", b, k, pls[b].l[k], lclass);
    const size_t need = align_up(solve_ws_layout(pls[b], TUCKER_FP32, nullptr, &wss[b]));
    if (off + need > ws_bytes) return fail(TUCKER_EWORKSPACE, "batch workspace %zu too small (item %d)", ws_bytes, b);
    solve_ws_layout(pls[b], TUCKER_FP32, (char*)ws + off, &wss[b]);
    off += need;
  }
  // header and phase records
  char* pb = (char*)plan;
  BatchHeader* h = (BatchHeader*)pb;
  h->magic = 0;  // valid only once every table is written
  h->capacity = capacity;
  h->order = d;
  h->q = q;
  h->lclass = lclass;
  h->nphases = (int32_t)recs.size();
  h->table_bytes = tb;
  h->ws = (char*)ws;
  PhaseRec* pr = (PhaseRec*)(pb + align_up(sizeof(BatchHeader)));
  char* img = pb + align_up(sizeof(BatchHeader)) + align_up(recs.size() * sizeof(PhaseRec));
  // tables: walk the phase sequence with the same (mode, step, role) bookkeeping
  size_t ip = 0;
  auto fill_phase = [&](int k, int t, int role) {
    PhaseRec& r = recs[ip++];
    int* hdr = (int*)(img + r.hdr_off);
    char* desc = img + r.desc_off;
    const size_t dsz = batch_desc_bytes((BatchKind)r.kind);
    hdr[0] = nitems;
    int64_t acc = 0;
    for (int b = 0; b < nitems; ++b) {
      hdr[1 + b] = (int)acc;
      acc += batch_desc((BatchKind)r.kind, k, t, role, pls[b], wss[b], items[b], shift, d, q,
                        desc + (size_t)b * dsz);
      batch_phase_work((BatchKind)r.kind, k, role, pls[b], &r.bytes, &r.flops);
    }
    hdr[1 + nitems] = (int)acc;
    for (int x = 0; x < 8; ++x) hdr[2 + nitems + x] = 0;  // claim counters, zero at every upload
    return acc < (1ll << 31);
  };
  bool ok = fill_phase(0, 0, 0);  // init
  for (int k = 0; k < d && ok; ++k) {
    for (int i = 0; i < 4; ++i) ok = ok && fill_phase(k, 0, 0);  // fill, cr, cr, reduce
    ok = ok && fill_phase(k, 0, 0);                                // gram
    for (int role = 0; role < 3; ++role) ok = ok && fill_phase(k, 0, role);
    ok = ok && fill_phase(k, 0, 0);                                // svd
    for (int t = 1; t <= q; ++t) {
      for (int i = 0; i < 5; ++i) ok = ok && fill_phase(k, t, 0);  // rc, rc, cr, cr, reduce
      ok = ok && fill_phase(k, t, 0);                              // gram
      for (int role = 0; role < 3; ++role) ok = ok && fill_phase(k, t, role);
      ok = ok && fill_phase(k, t, 0);                              // svd
    }
    ok = ok && fill_phase(k, q, 0);  // rotate
    ok = ok && fill_phase(k, q, 0);  // signfix
    ok = ok && fill_phase(k, q, 1);  // core (rows)
    ok = ok && fill_phase(k, q, 1);  // core (cols)
  }
  if (!ok) return fail(TUCKER_EUNSUPPORTED, "batch has more than 2^31 work items in a phase");
  if (ip != recs.size()) return fail(TUCKER_EINVAL, "internal: phase bookkeeping mismatch");
  for (size_t i = 0; i < recs.size(); ++i) pr[i] = recs[i];
  h->magic = kBatchMagic;
  return TUCKER_OK;
}

int tucker_batch_step(const void* plan, hipStream_t stream) {
  if (plan == nullptr) return fail(TUCKER_EINVAL, "plan is null");
  const char* pb = (const char*)plan;
  const BatchHeader* h = (const BatchHeader*)pb;
  if (h->magic != kBatchMagic) return fail(TUCKER_EINVAL, "not a batch plan");
  const PhaseRec* pr = (const PhaseRec*)(pb + align_up(sizeof(BatchHeader)));
  const char* img = pb + align_up(sizeof(BatchHeader)) + align_up((size_t)h->nphases * sizeof(PhaseRec));
  hipError_t e = hipMemcpyAsync(h->ws, img, h->table_bytes, hipMemcpyHostToDevice, stream);
  for (int i = 0; i < h->nphases && e == hipSuccess; ++i) {
    const BatchKind kind = (BatchKind)pr[i].kind;
    int* hdr = (int*)(h->ws + pr[i].hdr_off);
    const void* desc = h->ws + pr[i].desc_off;
    const bool orth = kind == BK_INIT || kind == BK_GRAM || kind == BK_PASS || kind == BK_SVD || kind == BK_ROTATE ||
                      kind == BK_SIGNFIX;
    if (orth) {
      e = launch_batch_orth(kind, h->lclass, hdr, desc, stream);
      continue;
    }
    const int cls = (kind == BK_CR_SPLIT || kind == BK_CR_COLS) ? KC_COLREDUCE
                    : (kind == BK_RC_SPLIT || kind == BK_RC_COLS) ? KC_ROWCONTRACT
                    : kind == BK_REDUCE ? KC_REDUCE : KC_FILL;
    TimingScope ts(cls, stream, pr[i].bytes, pr[i].flops, true);
    e = launch_batch_ttm(kind, h->lclass, hdr, desc, stream);
  }
  return dev_check(e, "batch step");
}

}  // extern "C"

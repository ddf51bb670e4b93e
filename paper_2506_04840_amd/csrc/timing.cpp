// Opt-in launch timing: when a kernel class is enabled, every launch of that
// class is timed by a pair of HIP events on the launch stream (recorded by the
// kernel dispatch itself for launches made through TK_LAUNCH, else around
// the launch), and its algorithmic bytes and flops are summed. Measurement only; the
// disabled path costs one relaxed atomic load per launch.
#include <atomic>
#include <mutex>
#include <vector>

#include "internal.hpp"
#include "tucker.h"

namespace tk {
namespace {

struct Slot {
  hipEvent_t a, b;
  double bytes, flops;
};

struct Timing {
  std::mutex mu;
  std::atomic<int> which{-1};
  std::vector<Slot> slots;
  size_t used = 0;
  size_t dropped = 0;
};

Timing& state() {
  static Timing t;
  return t;
}

}  // namespace

thread_local TimingScope* g_scope = nullptr;  // innermost active scope of this host thread

thread_local int g_fp32_products = TUCKER_FP32_SPLIT;
ProductScope::ProductScope(int fp32_products) : prev_(g_fp32_products) { g_fp32_products = fp32_products; }
ProductScope::~ProductScope() { g_fp32_products = prev_; }
bool fp32_split_products() { return g_fp32_products == TUCKER_FP32_SPLIT; }

TimingScope::TimingScope(int cls, hipStream_t st, double bytes, double flops, bool stamped)
    : slot_(-1), st_(st), stamped_(stamped), attached_(false), prev_(nullptr) {
  Timing& t = state();
  if (t.which.load(std::memory_order_relaxed) != cls) return;
  std::lock_guard<std::mutex> g(t.mu);
  if (t.which.load() != cls) return;
  if (t.used >= t.slots.size()) {
    ++t.dropped;
    return;
  }
  slot_ = (int)t.used++;
  Slot& s = t.slots[slot_];
  s.bytes = bytes;
  s.flops = flops;
  if (!stamped_) hipEventRecord(s.a, st_);  // else the TK_LAUNCH dispatch records both
  prev_ = g_scope;
  g_scope = this;
}

TimingScope::~TimingScope() {
  if (slot_ < 0) return;
  g_scope = prev_;
  if (attached_) return;
  Timing& t = state();
  std::lock_guard<std::mutex> g(t.mu);
  if (stamped_) hipEventRecord(t.slots[slot_].a, st_);  // nothing was launched: an empty interval
  hipEventRecord(t.slots[slot_].b, st_);
}

TimingScope* TimingScope::claim(hipStream_t st) {
  TimingScope* s = g_scope;
  if (s == nullptr || !s->stamped_ || s->attached_ || s->st_ != st) return nullptr;
  s->attached_ = true;
  return s;
}

hipEvent_t TimingScope::start() const { return state().slots[slot_].a; }
hipEvent_t TimingScope::stop() const { return state().slots[slot_].b; }

}  // namespace tk

using namespace tk;

extern "C" {

int tucker_timing_enable(int32_t kernel_class, int32_t capacity) {
  if (kernel_class < 0 || kernel_class >= KC_COUNT || capacity < 1 || capacity > (1 << 20)) return TUCKER_EINVAL;
  Timing& t = state();
  std::lock_guard<std::mutex> g(t.mu);
  for (Slot& s : t.slots) {
    hipEventDestroy(s.a);
    hipEventDestroy(s.b);
  }
  t.slots.clear();
  t.used = t.dropped = 0;
  t.slots.resize((size_t)capacity);
  for (Slot& s : t.slots) {
    if (hipEventCreate(&s.a) != hipSuccess || hipEventCreate(&s.b) != hipSuccess) {
      t.slots.clear();
      t.which.store(-1);
      return TUCKER_EDEVICE;
    }
  }
  t.which.store(kernel_class);
  return TUCKER_OK;
}

int tucker_timing_read(int32_t kernel_class, double* total_ms, int64_t* launches, double* bytes, double* flops) {
  Timing& t = state();
  std::lock_guard<std::mutex> g(t.mu);
  if (t.which.load() != kernel_class || total_ms == nullptr || launches == nullptr) return TUCKER_EINVAL;
  double ms = 0.0, by = 0.0, fl = 0.0;
  for (size_t i = 0; i < t.used; ++i) {
    Slot& s = t.slots[i];
    if (hipEventSynchronize(s.b) != hipSuccess) return TUCKER_EDEVICE;
    float e = 0.0f;
    if (hipEventElapsedTime(&e, s.a, s.b) != hipSuccess) return TUCKER_EDEVICE;
    ms += e;
    by += s.bytes;
    fl += s.flops;
  }
  *total_ms = ms;
  *launches = (int64_t)t.used;
  if (bytes) *bytes = by;
  if (flops) *flops = fl;
  return t.dropped ? TUCKER_EUNSUPPORTED : TUCKER_OK;
}

int tucker_timing_reset(void) {
  Timing& t = state();
  std::lock_guard<std::mutex> g(t.mu);
  t.used = t.dropped = 0;
  return TUCKER_OK;
}

int tucker_timing_disable(void) {
  Timing& t = state();
  std::lock_guard<std::mutex> g(t.mu);
  t.which.store(-1);
  for (Slot& s : t.slots) {
    hipEventDestroy(s.a);
    hipEventDestroy(s.b);
  }
  t.slots.clear();
  t.used = t.dropped = 0;
  return TUCKER_OK;
}

}  // extern "C"

// Host runtime of libbm: error state, device-memory pool, launch timing.
#include <cstdio>
#include <map>
#include <mutex>
#include <unordered_map>

#include "internal.hpp"

namespace bm {

// ------------------------------------------------------------------ errors

namespace {
thread_local std::string t_last_error;
}

void set_last_error(const std::string& s) { t_last_error = s; }
const char* last_error() { return t_last_error.c_str(); }

void fail(bm_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  throw Error{st, std::string(buf)};
}

// ------------------------------------------------------------------ memory
// Built-in caching pool: blocks are rounded up to size classes (256 B minimum,
// then quarter steps between powers of two) and kept per device after free, so
// repeated calls of the same shape allocate nothing from the runtime.  Frees
// are stream-ordered by construction: the library frees a block only after the
// call that used it has synchronised its stream.

namespace {

struct ExtAlloc {
  void* (*alloc)(size_t, void*, void*) = nullptr;
  void (*free_fn)(void*, void*, void*) = nullptr;
  void* ctx = nullptr;
};

std::mutex g_mu;
ExtAlloc g_ext;
std::multimap<std::pair<int, size_t>, void*> g_free;           // (device, size class) -> block
std::unordered_map<void*, std::pair<int, size_t>> g_used;      // block -> (device, size class)

size_t size_class(size_t n) {
  if (n <= 256) return 256;
  size_t p = 1;
  while (p < n) p <<= 1;
  const size_t q = p >> 3;  // eighth of the power of two
  size_t c = p >> 1;
  while (c < n) c += q;
  return c;
}

void release_all_locked() {
  for (auto& kv : g_free) (void)hipFree(kv.second);
  g_free.clear();
}

}  // namespace

void* dalloc(size_t bytes, hipStream_t s) {
  if (bytes == 0) return nullptr;
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_ext.alloc) {
    void* p = g_ext.alloc(bytes, (void*)s, g_ext.ctx);
    if (!p) fail(BM_ERR_OOM, "external allocator returned NULL for %zu bytes", bytes);
    g_used[p] = {-1, bytes};
    return p;
  }
  int dev = 0;
  BM_HIP(hipGetDevice(&dev));
  const size_t c = size_class(bytes);
  auto it = g_free.find({dev, c});
  if (it != g_free.end()) {
    void* p = it->second;
    g_free.erase(it);
    g_used[p] = {dev, c};
    return p;
  }
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, c);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    release_all_locked();
    e = hipMalloc(&p, c);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      fail(BM_ERR_OOM, "hipMalloc of %zu bytes failed", c);
    }
  }
  g_used[p] = {dev, c};
  return p;
}

void dfree(void* p, hipStream_t s) noexcept {
  if (!p) return;
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_used.find(p);
  if (it == g_used.end()) return;
  const auto key = it->second;
  g_used.erase(it);
  if (key.first < 0) {
    if (g_ext.free_fn) g_ext.free_fn(p, (void*)s, g_ext.ctx);
    return;
  }
  g_free.emplace(key, p);
}

bm_status set_allocator(void* (*alloc)(size_t, void*, void*), void (*free_fn)(void*, void*, void*),
                        void* ctx) {
  std::lock_guard<std::mutex> lk(g_mu);
  if ((alloc == nullptr) != (free_fn == nullptr)) {
    set_last_error("bm_set_allocator: alloc and free must both be set or both be NULL");
    return BM_ERR_INVALID_ARG;
  }
  if (!g_used.empty()) {
    set_last_error("bm_set_allocator: live allocations exist");
    return BM_ERR_INVALID_ARG;
  }
  release_all_locked();
  g_ext.alloc = alloc;
  g_ext.free_fn = free_fn;
  g_ext.ctx = ctx;
  return BM_OK;
}

void release_cached() {
  std::lock_guard<std::mutex> lk(g_mu);
  release_all_locked();
}

// ------------------------------------------------------------------ timing

// Timing events are reused: creating one costs more host time than recording
// it, and a call records a few dozen.  One pool per thread and device.
namespace {
thread_local std::map<int, std::vector<hipEvent_t>> t_events;

hipEvent_t take_event(int dev) {
  auto& v = t_events[dev];
  if (!v.empty()) {
    hipEvent_t e = v.back();
    v.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  BM_HIP(hipEventCreate(&e));
  return e;
}
}  // namespace

KTimer::KTimer(uint32_t kinds, hipStream_t s) : on_(kinds != 0), kinds_(kinds), s_(s) {
  if (on_) BM_HIP(hipGetDevice(&dev_));
}

KTimer::~KTimer() {
  auto& v = t_events[dev_];
  for (auto& r : recs_) {
    v.push_back(r.a);
    v.push_back(r.b);
  }
  if (cur_a_) v.push_back(cur_a_);
}

void KTimer::begin(int kind) {
  if (!on_) return;
  skip_ = !(kinds_ & (1u << kind));
  if (skip_) return;
  if (!cur_a_) cur_a_ = take_event(dev_);
  BM_HIP(hipEventRecord(cur_a_, s_));
  cur_kind_ = kind;
}

void KTimer::end(double bytes, double ops) {
  if (!on_ || skip_) return;
  hipEvent_t b = take_event(dev_);
  recs_.push_back(Rec{cur_kind_, cur_a_, b, bytes, ops});
  cur_a_ = nullptr;
  BM_HIP(hipEventRecord(b, s_));
}

void KTimer::set_last(double bytes, double ops) {
  if (!on_ || skip_ || recs_.empty()) return;
  recs_.back().bytes = bytes;
  recs_.back().ops = ops;
}

void KTimer::collect(bm_stats* st) {
  for (auto& r : recs_) {
    BM_HIP(hipEventSynchronize(r.b));
    float ms = 0;
    BM_HIP(hipEventElapsedTime(&ms, r.a, r.b));
    st->kernel_ms[r.kind] += ms;
    st->kernel_launches[r.kind] += 1;
    st->kernel_bytes[r.kind] += r.bytes;
    st->kernel_ops[r.kind] += r.ops;
  }
  auto& v = t_events[dev_];
  for (auto& r : recs_) {
    v.push_back(r.a);
    v.push_back(r.b);
  }
  recs_.clear();
}

// ------------------------------------------------------------------ devices

int cu_count() {
  static std::mutex mu;
  static std::map<int, int> cache;
  int dev = 0;
  BM_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(mu);
  auto it = cache.find(dev);
  if (it != cache.end()) return it->second;
  int n = 0;
  BM_HIP(hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev));
  if (n <= 0) n = 1;
  cache[dev] = n;
  return n;
}

bool is_device_ptr(const void* p) {
  if (!p) return false;
  hipPointerAttribute_t attr;
  hipError_t e = hipPointerGetAttributes(&attr, p);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return attr.type == hipMemoryTypeDevice || attr.type == hipMemoryTypeManaged;
}

}  // namespace bm

// kc_vaspace.hip -- device memory mapped at exactly the captured VAs.
//
// A replay restores captured bytes at the addresses they were captured at,
// so that pointers stored inside device memory stay valid.  In a fresh
// process that means reserving each captured address range before anything
// else allocates, backing it with device memory and enabling access; if a
// range cannot be placed at its address the replay must stop rather than run
// relocated.  HIP's virtual-memory calls give exactly that: an address
// reservation with a requested start, physical allocations mapped into it,
// and access rights per device.
#include <vector>

#include "kc_internal.h"

struct kc_vaspace {
  struct Span {
    uint64_t base = 0, size = 0;
    hipMemGenericAllocationHandle_t handle{};
    bool reserved = false, created = false, mapped = false;
  };
  int device = 0;
  std::vector<Span> spans;
};

namespace {

void release_all(kc_vaspace* vs) {
  for (auto it = vs->spans.rbegin(); it != vs->spans.rend(); ++it) {
    void* p = reinterpret_cast<void*>(it->base);
    if (it->mapped) (void)hipMemUnmap(p, it->size);
    if (it->created) (void)hipMemRelease(it->handle);
    if (it->reserved) (void)hipMemAddressFree(p, it->size);
    it->mapped = it->created = it->reserved = false;
  }
  (void)hipGetLastError();
}

// Granularity-aligned covers of the ranges, merged where they touch.
std::vector<kc_vaspace::Span> plan_spans(const kc_range* r, uint32_t n, uint64_t gran) {
  std::vector<kc_vaspace::Span> out;
  for (uint32_t i = 0; i < n; ++i) {
    const uint64_t lo = r[i].base / gran * gran;
    const uint64_t end = r[i].base + r[i].size;
    const uint64_t hi = (end + gran - 1) / gran * gran;
    if (!out.empty() && lo <= out.back().base + out.back().size) {
      const uint64_t cur = out.back().base + out.back().size;
      if (hi > cur) out.back().size = hi - out.back().base;
    } else {
      kc_vaspace::Span s;
      s.base = lo;
      s.size = hi - lo;
      out.push_back(s);
    }
  }
  return out;
}

}  // namespace

extern "C" {

int kc_vaspace_create(int hip_device, const kc_range* ranges, uint32_t n, kc_vaspace** out, uint32_t* n_spans,
                      uint64_t* mapped_bytes) {
  if (out == nullptr) return KC_EINVAL;
  *out = nullptr;
  const int st = kc_range_check(ranges, n, nullptr);
  if (st != KC_OK) return st;
  kc::DeviceGuard g(hip_device);
  if (!g.ok) return KC_EHIP;
  int vmm = 0;
  KC_HIP(hipDeviceGetAttribute(&vmm, hipDeviceAttributeVirtualMemoryManagementSupported, hip_device));
  if (!vmm) {
    kc::set_error_text("device has no virtual memory management");
    return KC_EHIP;
  }
  hipMemAllocationProp prop{};
  prop.type = hipMemAllocationTypePinned;
  prop.location.type = hipMemLocationTypeDevice;
  prop.location.id = hip_device;
  // Spans follow the recommended granularity (the runtime places reservations
  // of that size class where larger allocations go), at least the minimum.
  size_t gran = 0, rec = 0;
  KC_HIP(hipMemGetAllocationGranularity(&gran, &prop, hipMemAllocationGranularityMinimum));
  if (hipMemGetAllocationGranularity(&rec, &prop, hipMemAllocationGranularityRecommended) == hipSuccess && rec > gran)
    gran = rec;
  (void)hipGetLastError();
  if (gran == 0 || (gran & (gran - 1)) != 0) {
    kc::set_error_text("unexpected virtual memory granularity");
    return KC_EHIP;
  }
  kc_vaspace* vs = new (std::nothrow) kc_vaspace;
  if (vs == nullptr) return KC_ENOMEM;
  vs->device = hip_device;
  vs->spans = plan_spans(ranges, n, gran);
  uint64_t total = 0;
  for (auto& s : vs->spans) {
    void* want = reinterpret_cast<void*>(s.base);
    void* got = nullptr;
    hipError_t e = hipMemAddressReserve(&got, s.size, gran, want, 0);
    if (e != hipSuccess || got != want) {
      if (e == hipSuccess) (void)hipMemAddressFree(got, s.size);
      char msg[224];
      std::snprintf(msg, sizeof(msg), "span 0x%llx + 0x%llx (granularity 0x%llx) not reservable at its VA: %s 0x%llx",
                    (unsigned long long)s.base, (unsigned long long)s.size, (unsigned long long)gran,
                    e == hipSuccess ? "placed at" : hipGetErrorName(e), (unsigned long long)(uintptr_t)got);
      release_all(vs);
      delete vs;
      kc::set_error_text(msg);
      return KC_ERELOC;
    }
    s.reserved = true;
    if ((e = hipMemCreate(&s.handle, s.size, &prop, 0)) == hipSuccess) {
      s.created = true;
      if ((e = hipMemMap(want, s.size, 0, s.handle, 0)) == hipSuccess) {
        s.mapped = true;
        hipMemAccessDesc d{};
        d.location = prop.location;
        d.flags = hipMemAccessFlagsProtReadWrite;
        e = hipMemSetAccess(want, s.size, &d, 1);
      }
    }
    if (e != hipSuccess) {
      kc::set_error("hipMemCreate / hipMemMap / hipMemSetAccess", e);
      release_all(vs);
      delete vs;
      return e == hipErrorOutOfMemory ? KC_ENOMEM : KC_EHIP;
    }
    total += s.size;
  }
  if (n_spans) *n_spans = (uint32_t)vs->spans.size();
  if (mapped_bytes) *mapped_bytes = total;
  *out = vs;
  return KC_OK;
}

int kc_vaspace_suggest(int hip_device, uint64_t size, uint64_t* base) {
  if (base == nullptr || size == 0) return KC_EINVAL;
  *base = 0;
  kc::DeviceGuard g(hip_device);
  if (!g.ok) return KC_EHIP;
  hipMemAllocationProp prop{};
  prop.type = hipMemAllocationTypePinned;
  prop.location.type = hipMemLocationTypeDevice;
  prop.location.id = hip_device;
  size_t gran = 0, rec = 0;
  KC_HIP(hipMemGetAllocationGranularity(&gran, &prop, hipMemAllocationGranularityMinimum));
  if (hipMemGetAllocationGranularity(&rec, &prop, hipMemAllocationGranularityRecommended) == hipSuccess && rec > gran)
    gran = rec;
  (void)hipGetLastError();
  if (gran == 0) return KC_EHIP;
  const uint64_t span = (size + gran - 1) / gran * gran;
  // Where an unplaced reservation lands, then addresses well below it: the
  // runtime later claims blocks near the first placements for its own use, so
  // the first address below them that is granted exactly is the suggestion.
  void* p = nullptr;
  KC_HIP(hipMemAddressReserve(&p, span, gran, nullptr, 0));
  const uint64_t first = (uint64_t)(uintptr_t)p;
  KC_HIP(hipMemAddressFree(p, span));
  constexpr uint64_t kStep = 64ull << 30;
  for (uint64_t k = 1; k <= 8; ++k) {
    if (first < k * kStep + span) break;
    const uint64_t want = (first - k * kStep) / gran * gran;
    void* got = nullptr;
    if (hipMemAddressReserve(&got, span, gran, reinterpret_cast<void*>(want), 0) != hipSuccess) {
      (void)hipGetLastError();
      continue;
    }
    (void)hipMemAddressFree(got, span);
    if ((uint64_t)(uintptr_t)got == want) {
      *base = want;
      return KC_OK;
    }
  }
  *base = first;  // nothing below was granted exactly: the first placement
  return KC_OK;
}

void kc_vaspace_destroy(kc_vaspace* vs) {
  if (vs == nullptr) return;
  kc::DeviceGuard g(vs->device);
  (void)hipDeviceSynchronize();  // nothing may still write into the spans
  release_all(vs);
  delete vs;
}

}  // extern "C"

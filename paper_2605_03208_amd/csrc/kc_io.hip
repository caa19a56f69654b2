// kc_io.hip -- snapshot files: the packed snapshot streamed to host files
// through pinned chunk buffers (copies running ahead of the file writes), and
// loaded back for a restore.
#include <errno.h>
#include <fcntl.h>
#include <sys/stat.h>
#include <unistd.h>

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstring>
#include <string>
#include <thread>
#include <vector>

#include "kc_internal.h"

namespace kc {

// Pinned staging: kIoBufs chunk buffers, so that up to kIoBufs - 1 copies
// run ahead of the file reads or writes.
constexpr int kIoBufs = 4;
struct Pinned {
  uint8_t* p[kIoBufs] = {};
  hipEvent_t ev[kIoBufs] = {};
  ~Pinned() {
    for (int i = 0; i < kIoBufs; ++i) {
      if (ev[i]) (void)hipEventDestroy(ev[i]);
      if (p[i]) (void)hipHostFree(p[i]);
    }
  }
  hipError_t init(size_t bytes) {
    for (int i = 0; i < kIoBufs; ++i) {
      hipError_t e = hipHostMalloc(reinterpret_cast<void**>(&p[i]), bytes, hipHostMallocDefault);
      if (e != hipSuccess) return e;
      e = hipEventCreateWithFlags(&ev[i], hipEventDisableTiming);
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  }
};

// Where the host thread's time went: waiting for device copies, and inside
// file reads or writes.
struct IoClock {
  double copy_wait = 0.0, file = 0.0;
};

double now_s();

namespace {

bool write_all(int fd, const uint8_t* p, size_t n) {
  while (n > 0) {
    const ssize_t w = ::write(fd, p, n);
    if (w <= 0) return false;
    p += w;
    n -= (size_t)w;
  }
  return true;
}

bool read_all(int fd, uint8_t* p, size_t n) {
  while (n > 0) {
    const ssize_t r = ::read(fd, p, n);
    if (r <= 0) return false;
    p += r;
    n -= (size_t)r;
  }
  return true;
}

// [p, p + n) from the file at offset off, split into up to kIoThreads
// contiguous 1 MiB-aligned slices on as many threads: a page-cache copy runs at
// one core's memory bandwidth, and reads of one file proceed in parallel, so
// the slices' copies add up (2 GiB from a memory file system: 19-20 GB/s
// against 8.6-8.9 on one thread).  Writes stay on one thread: writes to one
// file take its inode lock in turn, and sliced writes measured no faster.  A
// thread that cannot be started has its slice read on the calling thread.
constexpr int kIoThreads = 4;
bool read_at(int fd, uint8_t* p, size_t n, uint64_t off) {
  const auto one = [fd, p, off](size_t a, size_t b) -> bool {
    while (a < b) {
      const ssize_t r = ::pread(fd, p + a, b - a, (off_t)(off + a));
      if (r <= 0) return false;
      a += (size_t)r;
    }
    return true;
  };
  const size_t slice = ((n + kIoThreads - 1) / kIoThreads + ((size_t)1 << 20) - 1) & ~(((size_t)1 << 20) - 1);
  if (n <= slice) return one(0, n);
  std::thread th[kIoThreads];
  bool ok[kIoThreads] = {};
  int k = 0;
  for (size_t a = slice; a < n; a += slice, ++k) {
    const size_t b = std::min(n, a + slice);
    try {
      th[k] = std::thread([&one, &ok, a, b, k] { ok[k] = one(a, b); });
    } catch (...) {
      ok[k] = one(a, b);
    }
  }
  bool all = one(0, slice);
  for (int i = 0; i < k; ++i) {
    if (th[i].joinable()) th[i].join();
    all = all && ok[i];
  }
  return all;
}

}  // namespace

// Device -> file in chunks: while chunk i is written, the copies of the
// next kIoBufs - 1 chunks are in flight.
int stream_to_file(const std::string& path, const void* src_d, uint64_t bytes, Pinned& pin, size_t chunk,
                   hipStream_t s, IoClock& ck, std::string& err) {
  const int fd = ::open(path.c_str(), O_WRONLY | O_CREAT | O_TRUNC, 0644);
  if (fd < 0) {
    err = "cannot create " + path;
    return KC_EINVAL;
  }
  const uint8_t* src = static_cast<const uint8_t*>(src_d);
  const uint64_t n_chunks = (bytes + chunk - 1) / chunk;
  uint64_t issued = 0;
  int st = KC_OK;
  for (uint64_t i = 0; i < n_chunks && st == KC_OK; ++i) {
    // chunk j goes to buffer j % kIoBufs, free once chunk j - kIoBufs has been written
    for (; issued < n_chunks && issued < i + kIoBufs; ++issued) {
      const uint64_t off = issued * chunk, len = std::min<uint64_t>(chunk, bytes - off);
      hipError_t e = hipMemcpyAsync(pin.p[issued % kIoBufs], src + off, len, hipMemcpyDeviceToHost, s);
      if (e == hipSuccess) e = hipEventRecord(pin.ev[issued % kIoBufs], s);
      if (e != hipSuccess) {
        err = std::string("D2H copy: ") + hipGetErrorName(e);
        st = KC_EHIP;
        break;
      }
    }
    if (st != KC_OK) break;
    const uint64_t off = i * chunk, len = std::min<uint64_t>(chunk, bytes - off);
    double t = now_s();
    hipError_t e = hipEventSynchronize(pin.ev[i % kIoBufs]);
    ck.copy_wait += now_s() - t;
    if (e != hipSuccess) {
      err = std::string("D2H wait: ") + hipGetErrorName(e);
      st = KC_EHIP;
      break;
    }
    t = now_s();
    const bool ok = write_all(fd, pin.p[i % kIoBufs], len);
    ck.file += now_s() - t;
    if (!ok) {
      err = "short write to " + path;
      st = KC_EINVAL;
    }
  }
  if (st != KC_OK) (void)hipStreamSynchronize(s);  // no copy may still target the staging buffers
  if (::close(fd) != 0 && st == KC_OK) {
    err = "close " + path;
    st = KC_EINVAL;
  }
  return st;
}

// File -> device in chunks: chunk i is read while the copies of the previous
// chunks (up to kIoBufs - 1) are in flight.
int stream_from_file(const std::string& path, void* dst_d, uint64_t bytes, Pinned& pin, size_t chunk,
                     hipStream_t s, IoClock& ck, std::string& err) {
  const int fd = ::open(path.c_str(), O_RDONLY);
  if (fd < 0) {
    err = "cannot open " + path;
    return KC_EINVAL;
  }
  struct stat stt;
  if (::fstat(fd, &stt) != 0 || (uint64_t)stt.st_size != bytes) {
    ::close(fd);
    err = path + ": size does not match the manifest";
    return KC_EINVAL;
  }
  uint8_t* dst = static_cast<uint8_t*>(dst_d);
  const uint64_t n_chunks = (bytes + chunk - 1) / chunk;
  int st = KC_OK;
  for (uint64_t i = 0; i < n_chunks && st == KC_OK; ++i) {
    const uint64_t off = i * chunk, len = std::min<uint64_t>(chunk, bytes - off);
    const int b = (int)(i % kIoBufs);
    if (i >= (uint64_t)kIoBufs) {  // the buffer's previous copy must have left it
      const double t = now_s();
      hipError_t e = hipEventSynchronize(pin.ev[b]);
      ck.copy_wait += now_s() - t;
      if (e != hipSuccess) {
        err = std::string("H2D wait: ") + hipGetErrorName(e);
        st = KC_EHIP;
        break;
      }
    }
    const double t = now_s();
    const bool ok = read_at(fd, pin.p[b], len, off);
    ck.file += now_s() - t;
    if (!ok) {
      err = "short read from " + path;
      st = KC_EINVAL;
      break;
    }
    hipError_t e = hipMemcpyAsync(dst + off, pin.p[b], len, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipEventRecord(pin.ev[b], s);
    if (e != hipSuccess) {
      err = std::string("H2D copy: ") + hipGetErrorName(e);
      st = KC_EHIP;
    }
  }
  ::close(fd);
  const double t = now_s();
  hipError_t e = hipStreamSynchronize(s);  // also on failure: no copy may still read the staging buffers
  ck.copy_wait += now_s() - t;
  if (st == KC_OK && e != hipSuccess) {
    err = std::string("H2D drain: ") + hipGetErrorName(e);
    st = KC_EHIP;
  }
  return st;
}

int write_text(const std::string& path, const std::string& text) {
  const int fd = ::open(path.c_str(), O_WRONLY | O_CREAT | O_TRUNC, 0644);
  if (fd < 0) return KC_EINVAL;
  const bool ok = write_all(fd, reinterpret_cast<const uint8_t*>(text.data()), text.size());
  return (::close(fd) == 0 && ok) ? KC_OK : KC_EINVAL;
}

int write_bytes(const std::string& path, const void* p, size_t n) {
  const int fd = ::open(path.c_str(), O_WRONLY | O_CREAT | O_TRUNC, 0644);
  if (fd < 0) return KC_EINVAL;
  const bool ok = write_all(fd, static_cast<const uint8_t*>(p), n);
  return (::close(fd) == 0 && ok) ? KC_OK : KC_EINVAL;
}

int read_bytes(const std::string& path, std::vector<uint8_t>& out) {
  const int fd = ::open(path.c_str(), O_RDONLY);
  if (fd < 0) return KC_EINVAL;
  struct stat stt;
  if (::fstat(fd, &stt) != 0) {
    ::close(fd);
    return KC_EINVAL;
  }
  out.resize((size_t)stt.st_size);
  const bool ok = read_all(fd, out.data(), out.size());
  ::close(fd);
  return ok ? KC_OK : KC_EINVAL;
}

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

}  // namespace kc

// ---------------------------------------------------------------------------
// extern "C" entry points
// ---------------------------------------------------------------------------
namespace {

struct FileHeader {  // header.bin: 64 bytes, little-endian
  char magic[8];     // "KCSNAP01"
  uint32_t version;
  uint32_t page_size;
  uint64_t seed;
  uint64_t n_ranges, n_pages, n_kept, n_packed;
  uint32_t delta, reserved;
};
static_assert(sizeof(FileHeader) == 64, "header layout");

constexpr uint64_t kDefaultChunk = 64ull << 20;  // the paper's default chunk size

std::string join(const char* dir, const char* name) { return std::string(dir) + "/" + name; }

}  // namespace

using namespace kc;

extern "C" {

int kc_snapshot_save(kc_ctx* c, const kc_rangeset* rs, const char* dir, uint64_t seed, const uint64_t* hash_d,
                     const uint64_t* zero_bm_d, const uint64_t* changed_bm_d, const void* packed_d,
                     const uint64_t* page_va_d, const uint64_t* n_kept_d, uint64_t cap_pages, uint64_t chunk_bytes,
                     void* stream, kc_io_stats* stats) {
  if (c == nullptr || rs == nullptr || rs->ctx != c || dir == nullptr || n_kept_d == nullptr) return KC_EINVAL;
  if (rs->n_pages > 0 && (hash_d == nullptr || zero_bm_d == nullptr)) return KC_EINVAL;
  if (cap_pages > 0 && (packed_d == nullptr || page_va_d == nullptr)) return KC_EINVAL;
  const uint64_t chunk = chunk_bytes ? chunk_bytes : kDefaultChunk;
  if (chunk < 4096 || chunk > (1ull << 32)) return KC_EINVAL;
  DeviceGuard g(c->device);
  if (!g.ok) return KC_EHIP;
  const hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const double t0 = now_s();
  if (::mkdir(dir, 0755) != 0 && errno != EEXIST) {
    set_error_text("cannot create the snapshot directory");
    return KC_EINVAL;
  }
  uint64_t n_kept = 0;
  KC_HIP(hipMemcpyAsync(&n_kept, n_kept_d, 8, hipMemcpyDeviceToHost, s));
  KC_HIP(hipStreamSynchronize(s));
  const uint64_t n_packed = std::min(n_kept, cap_pages);
  // metadata first, so a failure while streaming data leaves a readable manifest
  FileHeader h{};
  std::memcpy(h.magic, "KCSNAP01", 8);
  h.version = 1;
  h.page_size = 1u << rs->ushift;  // the hash unit: 4 KiB pages unless the range set was made with another
  h.seed = seed;
  h.n_ranges = rs->n_ranges;
  h.n_pages = rs->n_pages;
  h.n_kept = n_kept;
  h.n_packed = n_packed;
  h.delta = changed_bm_d != nullptr ? 1u : 0u;
  std::string js = "{\n  \"format\": \"kc-snapshot\",\n  \"version\": 1,\n";
  char buf[256];
  std::snprintf(buf, sizeof(buf), "  \"page_size\": %u,\n", h.page_size);
  js += buf;
  std::snprintf(buf, sizeof(buf),
                "  \"seed\": %llu,\n  \"n_ranges\": %llu,\n  \"n_pages\": %llu,\n  \"n_kept\": %llu,\n"
                "  \"n_packed\": %llu,\n  \"delta\": %s,\n  \"chunk_bytes\": %llu,\n  \"regions\": [\n",
                (unsigned long long)seed, (unsigned long long)rs->n_ranges, (unsigned long long)rs->n_pages,
                (unsigned long long)n_kept, (unsigned long long)n_packed, h.delta ? "true" : "false",
                (unsigned long long)chunk);
  js += buf;
  for (uint32_t i = 0; i < rs->n_ranges; ++i) {
    std::snprintf(buf, sizeof(buf), "    {\"base\": \"0x%llx\", \"size\": %llu}%s\n",
                  (unsigned long long)rs->host_ranges[i].base, (unsigned long long)rs->host_ranges[i].size,
                  i + 1 < rs->n_ranges ? "," : "");
    js += buf;
  }
  js += "  ],\n  \"files\": [\"header.bin\", \"ranges.bin\", \"hash.bin\", \"zero_bm.bin\"";
  js += h.delta ? ", \"changed_bm.bin\"" : "";
  js += ", \"page_va.bin\", \"packed.bin\"]\n}\n";
  if (write_text(join(dir, "manifest.json"), js) != KC_OK ||
      write_bytes(join(dir, "header.bin"), &h, sizeof(h)) != KC_OK ||
      write_bytes(join(dir, "ranges.bin"), rs->host_ranges.data(), sizeof(kc_range) * rs->n_ranges) != KC_OK) {
    set_error_text("cannot write the snapshot metadata");
    return KC_EINVAL;
  }
  Pinned pin;
  KC_HIP(pin.init(chunk));
  IoClock ck;
  std::string err;
  struct Part {
    const char* name;
    const void* src;
    uint64_t bytes;
  } parts[] = {{"hash.bin", hash_d, 8 * rs->n_pages},
               {"zero_bm.bin", zero_bm_d, 8 * rs->n_words},
               {"changed_bm.bin", changed_bm_d, changed_bm_d ? 8 * rs->n_words : 0},
               {"page_va.bin", page_va_d, 8 * n_packed},
               {"packed.bin", packed_d, (n_packed << rs->ushift)}};
  uint64_t total = 0;
  for (const Part& p : parts) {
    if (p.src == nullptr && std::strcmp(p.name, "changed_bm.bin") == 0) continue;
    const int st = stream_to_file(join(dir, p.name), p.src, p.bytes, pin, chunk, s, ck, err);
    if (st != KC_OK) {
      set_error_text(err.c_str());
      return st;
    }
    total += p.bytes;
  }
  if (stats) {
    stats->bytes = total;
    stats->seconds = now_s() - t0;
    stats->copy_wait_s = ck.copy_wait;
    stats->file_s = ck.file;
  }
  return KC_OK;
}

int kc_snapshot_load(kc_ctx* c, const kc_rangeset* rs, const char* dir, uint64_t* hash_d, uint64_t* zero_bm_d,
                     uint64_t* changed_bm_d, void* packed_d, uint64_t* page_va_d, uint64_t* n_kept_d,
                     uint64_t cap_pages, uint64_t chunk_bytes, void* stream, kc_io_stats* stats) {
  if (c == nullptr || rs == nullptr || rs->ctx != c || dir == nullptr || n_kept_d == nullptr) return KC_EINVAL;
  if (rs->n_pages > 0 && zero_bm_d == nullptr) return KC_EINVAL;
  const uint64_t chunk = chunk_bytes ? chunk_bytes : kDefaultChunk;
  if (chunk < 4096 || chunk > (1ull << 32)) return KC_EINVAL;
  DeviceGuard g(c->device);
  if (!g.ok) return KC_EHIP;
  const hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const double t0 = now_s();
  std::vector<uint8_t> hb, rb;
  if (read_bytes(join(dir, "header.bin"), hb) != KC_OK || hb.size() != sizeof(FileHeader)) {
    set_error_text("missing or short header.bin");
    return KC_EINVAL;
  }
  FileHeader h;
  std::memcpy(&h, hb.data(), sizeof(h));
  if (std::memcmp(h.magic, "KCSNAP01", 8) != 0 || h.version != 1) {
    set_error_text("not a snapshot directory of this format");
    return KC_EINVAL;
  }
  if (h.page_size != (1u << rs->ushift)) {
    set_error_text("the snapshot's hash unit differs from the range set's");
    return KC_EINVAL;
  }
  // the snapshot must describe exactly this range set (same VAs, same sizes)
  if (read_bytes(join(dir, "ranges.bin"), rb) != KC_OK || h.n_ranges != rs->n_ranges || h.n_pages != rs->n_pages ||
      rb.size() != sizeof(kc_range) * rs->n_ranges ||
      (rs->n_ranges && std::memcmp(rb.data(), rs->host_ranges.data(), rb.size()) != 0)) {
    set_error_text("snapshot ranges differ from the range set");
    return KC_EINVAL;
  }
  if (h.n_kept > h.n_pages || h.n_packed > h.n_kept) {
    set_error_text("inconsistent snapshot header: kept or packed page count out of range");
    return KC_EINVAL;
  }
  if (h.n_packed < h.n_kept) {  // saved with a capacity below its kept count: pages would stay unrestored
    set_error_text("the snapshot was saved truncated (fewer packed pages than kept pages)");
    return KC_ELIMIT;
  }
  if (h.n_packed > cap_pages) {
    set_error_text("more packed pages than cap_pages");
    return KC_ELIMIT;
  }
  if (h.n_packed > 0 && (packed_d == nullptr || page_va_d == nullptr)) return KC_EINVAL;
  if (h.delta && changed_bm_d == nullptr) return KC_EINVAL;
  Pinned pin;
  KC_HIP(pin.init(chunk));
  IoClock ck;
  std::string err;
  struct Part {
    const char* name;
    void* dst;
    uint64_t bytes;
  } parts[] = {{"hash.bin", hash_d, 8 * rs->n_pages},
               {"zero_bm.bin", zero_bm_d, 8 * rs->n_words},
               {"changed_bm.bin", h.delta ? changed_bm_d : nullptr, 8 * rs->n_words},
               {"page_va.bin", page_va_d, 8 * h.n_packed},
               {"packed.bin", packed_d, (h.n_packed << rs->ushift)}};
  uint64_t total = 0;
  for (const Part& p : parts) {
    if (p.dst == nullptr || p.bytes == 0) continue;
    const int st = stream_from_file(join(dir, p.name), p.dst, p.bytes, pin, chunk, s, ck, err);
    if (st != KC_OK) {
      set_error_text(err.c_str());
      return st;
    }
    total += p.bytes;
  }
  KC_HIP(hipMemcpyAsync(n_kept_d, &h.n_kept, 8, hipMemcpyHostToDevice, s));
  KC_HIP(hipStreamSynchronize(s));
  if (stats) {
    stats->bytes = total;
    stats->seconds = now_s() - t0;
    stats->copy_wait_s = ck.copy_wait;
    stats->file_s = ck.file;
  }
  return KC_OK;
}

}  // extern "C"

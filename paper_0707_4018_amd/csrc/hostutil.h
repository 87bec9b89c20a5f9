// Host-side helpers shared by the library's translation units: error
// propagation (exceptions inside, status codes at the C ABI) and owned
// device buffers.
#pragma once
#include <hip/hip_runtime.h>

#include <string>

#include "amg.h"

namespace amg {
namespace host {

std::string& last_error();

struct Fail {
  amg_status s;
  std::string msg;
};

[[noreturn]] inline void fail(amg_status s, const std::string& m) { throw Fail{s, m}; }

inline void hip_check(hipError_t e, const char* what) {
  if (e != hipSuccess) fail(AMG_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}
#define HIPC(x) hip_check((x), #x)

// Owned device allocation.
// Where the device buffers of every handle come from: hipMalloc / hipFree,
// or a caller's pair of routines (amg_set_allocator).  Process-wide.
struct Allocator {
  void* (*alloc)(size_t, void*, void*) = nullptr;
  void (*release)(void*, void*, void*) = nullptr;
  void* ctx = nullptr;
};
inline Allocator& allocator() {
  static Allocator a;
  return a;
}

struct Buf {
  void* p = nullptr;
  size_t bytes = 0;
  Allocator owner;  // the routines that made p (released through the same ones)
  Buf() = default;
  Buf(const Buf&) = delete;
  Buf& operator=(const Buf&) = delete;
  Buf(Buf&& o) noexcept : p(o.p), bytes(o.bytes), owner(o.owner) { o.p = nullptr; o.bytes = 0; }
  ~Buf() { release(); }
  void release() {
    if (p) {
      if (owner.release) {
        // a caching allocator hands the block out again at once: no kernel
        // queued on any stream may still use it (what hipFree guarantees)
        (void)hipDeviceSynchronize();
        owner.release(p, nullptr, owner.ctx);
      } else {
        (void)hipFree(p);
      }
    }
    p = nullptr;
    bytes = 0;
  }
  void ensure(size_t n) {
    if (n <= bytes && p) return;
    release();
    if (n == 0) n = 16;
    const Allocator a = allocator();
    if (a.alloc) {
      p = a.alloc(n, nullptr, a.ctx);
      if (p == nullptr) fail(AMG_ERR_NOMEM, "allocator returned no memory for " + std::to_string(n) + " bytes");
    } else if (hipMalloc(&p, n) != hipSuccess) {
      p = nullptr;
      fail(AMG_ERR_NOMEM, "hipMalloc of " + std::to_string(n) + " bytes failed");
    }
    owner = a;
    bytes = n;
  }
  template <typename T> T* as() const { return reinterpret_cast<T*>(p); }
};


}  // namespace host
}  // namespace amg

// C ABI wrappers: exceptions become status codes and a thread-local message
#define AMG_TRY try {
#define AMG_CATCH                                              \
  }                                                            \
  catch (const Fail& f) {                                      \
    last_error() = f.msg;                                      \
    return f.s;                                                \
  }                                                            \
  catch (const std::exception& e) {                            \
    last_error() = e.what();                                   \
    return AMG_ERR_HIP;                                        \
  }                                                            \
  return AMG_OK;


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
struct Buf {
  void* p = nullptr;
  size_t bytes = 0;
  Buf() = default;
  Buf(const Buf&) = delete;
  Buf& operator=(const Buf&) = delete;
  Buf(Buf&& o) noexcept : p(o.p), bytes(o.bytes) { o.p = nullptr; o.bytes = 0; }
  ~Buf() { release(); }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
  void ensure(size_t n) {
    if (n <= bytes && p) return;
    release();
    if (n == 0) n = 16;
    if (hipMalloc(&p, n) != hipSuccess) {
      p = nullptr;
      fail(AMG_ERR_NOMEM, "hipMalloc of " + std::to_string(n) + " bytes failed");
    }
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


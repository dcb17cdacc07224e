// Shared host-side infrastructure of the pbmp library: error type, device
// buffers, and the declarations of every kernel launcher.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <stdexcept>
#include <string>
#include <utility>
#include <vector>

#include "../../include/pbmp.h"

namespace pbmp {

struct Error : std::runtime_error {
  int code;
  Error(int c, const std::string &m) : std::runtime_error(m), code(c) {}
};

#define PBMP_HIP(x)                                                          \
  do {                                                                       \
    hipError_t pbmp_err_ = (x);                                                     \
    if (pbmp_err_ != hipSuccess)                                                  \
      throw ::pbmp::Error(PBMP_EHIP, std::string(#x) + ": " +               \
                                         hipGetErrorString(pbmp_err_));             \
  } while (0)

#define PBMP_REQUIRE(cond, code, msg)                                       \
  do {                                                                       \
    if (!(cond)) throw ::pbmp::Error((code), (msg));                         \
  } while (0)

// Owning device buffer (hipMalloc / hipFree), move-only.
template <class T> struct Dbuf {
  T *p = nullptr;
  size_t n = 0;
  Dbuf() = default;
  Dbuf(const Dbuf &) = delete;
  Dbuf &operator=(const Dbuf &) = delete;
  ~Dbuf() { release(); }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    n = 0;
  }
  void alloc(size_t count) {
    if (count == n && p) return;
    release();
    if (count == 0) return;
    hipError_t e = hipMalloc(reinterpret_cast<void **>(&p), count * sizeof(T));
    if (e != hipSuccess) {
      p = nullptr;
      (void)hipGetLastError();
      throw Error(PBMP_ENOMEM, "hipMalloc of " +
                                   std::to_string(count * sizeof(T)) +
                                   " bytes failed");
    }
    n = count;
  }
  void swap(Dbuf &o) {
    std::swap(p, o.p);
    std::swap(n, o.n);
  }
  // grow-only allocation for scratch buffers
  void reserve(size_t count) {
    if (count > n) alloc(count);
  }
  void upload(const T *h, size_t count, hipStream_t s) {
    alloc(count);
    if (count)
      PBMP_HIP(hipMemcpyAsync(p, h, count * sizeof(T), hipMemcpyHostToDevice, s));
  }
  void download(T *h, size_t count, hipStream_t s) const {
    if (count)
      PBMP_HIP(hipMemcpyAsync(h, p, count * sizeof(T), hipMemcpyDeviceToHost, s));
  }
  void zero(hipStream_t s) {
    if (n) PBMP_HIP(hipMemsetAsync(p, 0, n * sizeof(T), s));
  }
};

// ---------------------------------------------------------------- rules
// Triangle rule in barycentric coordinates, weights summing to 1.
struct TriRule {
  int n = 0;
  double b[19][3];
  double w[19];
};
TriRule far_rule(int k);  // 1 (centroid) or 3 (interior degree-2 rule)
TriRule near_rule19();    // symmetric degree-9 rule from its moment equations
void gauss_legendre(int n, double *x, double *w);  // nodes/weights on [-1,1]

// Rule data passed by value to kernels.
struct RuleArgs {
  int nf, nn, ngl;
  double fb[3][3], fw[3];     // far rule (up to 3 nodes)
  double nb[19][3], nw[19];   // near rule
  double glx[32], glw[32];    // edge rule for singular panels
};

}  // namespace pbmp

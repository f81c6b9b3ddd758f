// Shared definitions of the RT-CCSD HIP library (gfx950).
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>
#include <cstdio>
#include <stdexcept>
#include <string>

namespace rtcc {

// Thrown inside the library and turned into a status code at the C boundary.
struct Error : std::runtime_error {
  int code;
  Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

constexpr int kOk = 0, kEInval = -1, kENoMem = -2, kEHip = -3, kENonFinite = -4, kENotConv = -5;

#define RTCC_HIP(call)                                                                 \
  do {                                                                                 \
    hipError_t e_ = (call);                                                            \
    if (e_ != hipSuccess)                                                              \
      throw ::rtcc::Error(::rtcc::kEHip, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

#define RTCC_CHECK(cond, code, msg)                         \
  do {                                                      \
    if (!(cond)) throw ::rtcc::Error((code), (msg));        \
  } while (0)

inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Message of a failed call that has no context (read with rtcc_last_error(NULL)).
void set_noctx_error(const std::string& msg);

}  // namespace rtcc

// Kernels compiled at run time (the ROCm installation's hipRTC) for one
// structure of input, such as
// the tiled channel kernel specialised to a channel's plan.  A compiled
// kernel is cached for the process by (device, source text, entry name), so
// objects with the same structure share one code object; code objects stay
// loaded until the process ends.
#pragma once

#include <hip/hip_runtime.h>

#include <string>

namespace qcw {

struct RtcKernel {
  hipFunction_t fn;
  int num_regs;  // VGPRs per lane
};

// Compiles `src` for the current device (once per device, source and name;
// thread-safe) and sets *out to its function `name`.  QCW_OK, or QCW_EHIP
// with the compiler's log in the thread's last error.
int rtc_get(const std::string &src, const char *name, const RtcKernel **out);
// Compiles `src` without loading it (no device needed): the code object's size.
int rtc_compile(const std::string &src, const char *name, size_t *code_bytes);
// The run-time compiler's version, major * 100 + minor (0: not available).
int rtc_compiler_version();

}  // namespace qcw

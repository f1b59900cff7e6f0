// Host-side internals shared by the library's translation units: error state,
// argument validation, gate geometry and kernel timing.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "qcw.h"
#include "qcw_common.h"

namespace qcw {

// Checks that [ptr, ptr + bytes) lies inside one device allocation.
int check_device_range(const void *ptr, uint64_t bytes, const char *what);

// Kernel timing (see qcw_timing_* in qcw.h).
bool timing_on();
struct TimedLaunch {
  TimedLaunch(int family, hipStream_t s);
  ~TimedLaunch();
  int family;
  hipStream_t stream;
  hipEvent_t e0 = nullptr, e1 = nullptr;
};

// Launchers (sweep.hip).
int launch_sweep(const Geom &g, const qcw_c64 *U, const qcw_c64 *in, qcw_c64 *out,
                 hipStream_t s);
int launch_pick(const Geom &g, uint64_t *labels_dev, hipStream_t s);
// Fused passes (fused.hip).
int run_fused(qcw_c64 *psi, int nq, const qcw_gate *gates, int ngates, const qcw_c64 *mats,
              int tile_bits, int low_bits, int threads, hipStream_t s);
int fused_pass_count(int nq, const qcw_gate *gates, int ngates, int tile_bits, int low_bits);

}  // namespace qcw

// Host-side internals shared by the library's translation units: error state,
// argument validation, gate geometry and kernel timing.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "qcw.h"

namespace qcw {

constexpr int kMaxQubits = 34;

// Thread-local error text; returns `code` so callers can `return fail(...)`.
int fail(int code, const char *fmt, ...);
void clear_error();

// Geometry of one k-qubit gate on an nq-qubit state.
struct Geom {
  int k = 0;
  int nq = 0;
  int bit[3] = {0, 0, 0};  // bit position of each target, argument order
  int sb[3] = {0, 0, 0};   // the same positions sorted ascending
  uint64_t off[8] = {};    // label offset of local index r from the group base
};

// Validates nq, k and the targets (1-based, distinct, <= nq) and fills g.
int make_geom(int nq, int k, const int *targets, Geom *g);

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

}  // namespace qcw

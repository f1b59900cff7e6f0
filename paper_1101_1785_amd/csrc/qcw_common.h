// Host-only helpers shared by every translation unit (no HIP dependency):
// thread-local error text and gate-geometry validation.
#pragma once

#include <stdint.h>

#include "qcw.h"

namespace qcw {

constexpr int kMaxQubits = 34;

// Records a thread-local error text; returns `code` so callers can
// `return fail(...)`.
int fail(int code, const char *fmt, ...);
void clear_error();
const char *last_error();

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

}  // namespace qcw

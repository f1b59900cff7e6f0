// Error state and gate geometry (host only).
#include <stdarg.h>
#include <stdio.h>

#include <algorithm>

#include "qcw_common.h"

namespace qcw {

static thread_local char g_err[512];

int fail(int code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  snprintf(g_err, sizeof(g_err), "%s", buf);
  return code;
}

void clear_error() { g_err[0] = 0; }

const char *last_error() { return g_err; }

int make_geom(int nq, int k, const int *targets, Geom *g) {
  if (nq < 1 || nq > kMaxQubits) return fail(QCW_EINVAL, "nq=%d outside [1, %d]", nq, kMaxQubits);
  if (k < 1 || k > 3) return fail(QCW_EINVAL, "k=%d outside {1, 2, 3}", k);
  if (k > nq) return fail(QCW_EINVAL, "k=%d exceeds nq=%d", k, nq);
  if (!targets) return fail(QCW_EINVAL, "targets is NULL");
  for (int j = 0; j < k; ++j) {
    if (targets[j] < 1 || targets[j] > nq)
      return fail(QCW_EINVAL, "target %d outside [1, %d]", targets[j], nq);
    for (int i = 0; i < j; ++i)
      if (targets[i] == targets[j]) return fail(QCW_EINVAL, "target %d repeated", targets[j]);
  }
  g->k = k;
  g->nq = nq;
  for (int j = 0; j < 3; ++j) g->bit[j] = g->sb[j] = 0;
  for (int j = 0; j < k; ++j) g->bit[j] = g->sb[j] = nq - targets[j];
  std::sort(g->sb, g->sb + k);
  // Member r: the first listed target is the most significant bit of r.
  for (int r = 0; r < (1 << k); ++r) {
    uint64_t o = 0;
    for (int j = 0; j < k; ++j)
      if ((r >> (k - 1 - j)) & 1) o |= (uint64_t)1 << g->bit[j];
    g->off[r] = o;
  }
  return QCW_OK;
}

}  // namespace qcw

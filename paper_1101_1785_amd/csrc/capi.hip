// C ABI entry points of the plain (one sweep per gate) path, argument
// validation, error reporting and kernel timing.
#include <hip/hip_runtime.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <vector>

#include "qcw_host.h"

namespace qcw {

int check_device_range(const void *ptr, uint64_t bytes, const char *what) {
  if (!ptr) return fail(QCW_EINVAL, "%s is NULL", what);
  hipPointerAttribute_t attr;
  hipError_t e = hipPointerGetAttributes(&attr, ptr);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(QCW_EINVAL, "%s is not a device pointer (%s)", what, hipGetErrorString(e));
  }
  if (attr.type != hipMemoryTypeDevice && attr.type != hipMemoryTypeManaged)
    return fail(QCW_EINVAL, "%s is not device memory", what);
  hipDeviceptr_t base = nullptr;
  size_t size = 0;
  e = hipMemGetAddressRange(&base, &size, (hipDeviceptr_t)ptr);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(QCW_EINVAL, "%s: cannot find its allocation (%s)", what, hipGetErrorString(e));
  }
  const uint64_t lo = (uint64_t)(uintptr_t)base, p = (uint64_t)(uintptr_t)ptr;
  if (p + bytes > lo + (uint64_t)size || p < lo)
    return fail(QCW_EINVAL, "%s: %llu bytes from this pointer overrun its allocation", what,
                (unsigned long long)bytes);
  return QCW_OK;
}

// ------------------------------------------------------------------ timing
namespace {
struct TimingState {
  std::mutex mu;
  bool on = false;
  struct Rec {
    int family;
    hipEvent_t e0, e1;
  };
  std::vector<Rec> pending;
  std::vector<hipEvent_t> pool;
  int64_t launches[QCW_KERNEL_COUNT] = {};
  double ms[QCW_KERNEL_COUNT] = {};
};
TimingState &ts() {
  static TimingState s;
  return s;
}
hipEvent_t take_event(TimingState &s) {
  if (!s.pool.empty()) {
    hipEvent_t e = s.pool.back();
    s.pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}
// Folds completed records into the totals (synchronising each).
void drain(TimingState &s) {
  for (auto &r : s.pending) {
    float ms = 0.f;
    if (hipEventSynchronize(r.e1) == hipSuccess && hipEventElapsedTime(&ms, r.e0, r.e1) == hipSuccess) {
      s.launches[r.family] += 1;
      s.ms[r.family] += ms;
    }
    s.pool.push_back(r.e0);
    s.pool.push_back(r.e1);
  }
  s.pending.clear();
}
}  // namespace

bool timing_on() { return ts().on; }

TimedLaunch::TimedLaunch(int fam, hipStream_t s) : family(fam), stream(s) {
  TimingState &t = ts();
  if (!t.on) return;
  std::lock_guard<std::mutex> lk(t.mu);
  e0 = take_event(t);
  e1 = take_event(t);
  if (e0 && e1) (void)hipEventRecord(e0, s);
}

TimedLaunch::~TimedLaunch() {
  if (!e0 || !e1) return;
  TimingState &t = ts();
  std::lock_guard<std::mutex> lk(t.mu);
  (void)hipEventRecord(e1, stream);
  t.pending.push_back({family, e0, e1});
  if (t.pending.size() > 4096) drain(t);
}

}  // namespace qcw

using namespace qcw;

extern "C" {

const char *qcw_strerror(int code) {
  switch (code) {
    case QCW_OK: return "ok";
    case QCW_EINVAL: return "invalid argument";
    case QCW_ENOMEM: return "out of memory";
    case QCW_EHIP: return "HIP runtime error";
    case QCW_EAGAIN: return "not ready";
  }
  return "unknown error";
}

const char *qcw_last_error(void) { return last_error(); }

int qcw_version(void) { return 200; }  // 0.2.0: compiled channel kernels, one-call and observed steps

int qcw_opk_to(int k, const int *targets, const qcw_c64 *U, const qcw_c64 *psi_in,
               qcw_c64 *psi_out, int nq, void *stream) {
  clear_error();
  Geom g;
  int rc = make_geom(nq, k, targets, &g);
  if (rc) return rc;
  if (!U) return fail(QCW_EINVAL, "matrix is NULL");
  if (!psi_in || !psi_out) return fail(QCW_EINVAL, "state pointer is NULL");
  const uint64_t bytes = ((uint64_t)1 << nq) * sizeof(qcw_c64);
  const uint64_t a = (uint64_t)(uintptr_t)psi_in, b = (uint64_t)(uintptr_t)psi_out;
  if (a != b && a < b + bytes && b < a + bytes)
    return fail(QCW_EINVAL, "psi_in and psi_out partially overlap");
  if ((rc = check_device_range(psi_in, bytes, "psi_in"))) return rc;
  if (a != b && (rc = check_device_range(psi_out, bytes, "psi_out"))) return rc;
  return launch_sweep(g, U, psi_in, psi_out, (hipStream_t)stream);
}

int qcw_opk(int k, const int *targets, const qcw_c64 *U, qcw_c64 *psi, int nq, void *stream) {
  return qcw_opk_to(k, targets, U, psi, psi, nq, stream);
}

int qcw_op1(const qcw_c64 *U, int is, qcw_c64 *psi, int nq, void *stream) {
  int t[1] = {is};
  return qcw_opk(1, t, U, psi, nq, stream);
}

int qcw_op2(const qcw_c64 *V, int is1, int is2, qcw_c64 *psi, int nq, void *stream) {
  int t[2] = {is1, is2};
  return qcw_opk(2, t, V, psi, nq, stream);
}

int qcw_op3(const qcw_c64 *W, int is1, int is2, int is3, qcw_c64 *psi, int nq, void *stream) {
  int t[3] = {is1, is2, is3};
  return qcw_opk(3, t, W, psi, nq, stream);
}

// OmegaALL runs as fused passes from this many qubits on (a pass then moves at
// least 64 MiB, so the plan's one-off synchronisation is small beside the
// sweeps it saves); tile shape as qcw_circuit_fused's default.
constexpr int kOmegaFusedMinQubits = 22;
constexpr int kOmegaTileBits = 12;
constexpr int kOmegaLowBits = 4;

int qcw_omega_all(const qcw_c64 *U, qcw_c64 *psi, int nq, void *stream) {
  clear_error();
  if (!U) return fail(QCW_EINVAL, "matrix is NULL");
  if (nq < 1 || nq > kMaxQubits) return fail(QCW_EINVAL, "nq=%d outside [1, %d]", nq, kMaxQubits);
  int rc = check_device_range(psi, ((uint64_t)1 << nq) * sizeof(qcw_c64), "psi");
  if (rc) return rc;
  if (nq >= kOmegaFusedMinQubits) {
    // the nq one-qubit gates as list-order fused passes: bit for bit the
    // sweeps below, in ~nq/8 passes over HBM instead of nq
    std::vector<qcw_gate> gl((size_t)nq);
    for (int q = 1; q <= nq; ++q) {
      qcw_gate &g = gl[q - 1];
      memset(&g, 0, sizeof g);
      g.k = 1;
      g.q[0] = q;
      g.mat = 0;
    }
    return run_fused(psi, nq, gl.data(), nq, U, kOmegaTileBits, kOmegaLowBits, 0, 0,
                     (hipStream_t)stream);
  }
  for (int q = 1; q <= nq; ++q) {
    Geom g;
    if ((rc = make_geom(nq, 1, &q, &g))) return rc;
    if ((rc = launch_sweep(g, U, psi, psi, (hipStream_t)stream))) return rc;
  }
  return QCW_OK;
}

int qcw_circuit(qcw_c64 *psi, int nq, const qcw_gate *gates, int ngates, const qcw_c64 *mats,
                int64_t nmats, void *stream) {
  clear_error();
  if (nq < 1 || nq > kMaxQubits) return fail(QCW_EINVAL, "nq=%d outside [1, %d]", nq, kMaxQubits);
  if (ngates < 0) return fail(QCW_EINVAL, "ngates < 0");
  if (ngates > 0 && (!gates || !mats)) return fail(QCW_EINVAL, "gates or mats is NULL");
  // Validate the whole circuit before launching anything.
  std::vector<Geom> geo((size_t)ngates);
  for (int i = 0; i < ngates; ++i) {
    int rc = make_geom(nq, gates[i].k, gates[i].q, &geo[i]);
    if (rc) {
      char why[512];
      snprintf(why, sizeof(why), "%s", last_error());
      return fail(rc, "gate %d: %s", i, why);
    }
    const int64_t mm = (int64_t)1 << (2 * gates[i].k);
    if (gates[i].mat < 0 || gates[i].mat + mm > nmats)
      return fail(QCW_EINVAL, "gate %d: matrix offset outside mats", i);
  }
  int rc = check_device_range(psi, ((uint64_t)1 << nq) * sizeof(qcw_c64), "psi");
  if (rc) return rc;
  if (nq <= kSmallMaxQubits)
    return run_small_circuit(psi, nq, geo.data(), gates, ngates, mats, (hipStream_t)stream);
  for (int i = 0; i < ngates; ++i)
    if ((rc = launch_sweep(geo[i], mats + gates[i].mat, psi, psi, (hipStream_t)stream))) return rc;
  return QCW_OK;
}

int qcw_debug_pick_device(int nq, int k, const int *targets, uint64_t *out_host) {
  clear_error();
  if (nq > 26) return fail(QCW_EINVAL, "nq=%d above the test limit 26", nq);
  Geom g;
  int rc = make_geom(nq, k, targets, &g);
  if (rc) return rc;
  if (!out_host) return fail(QCW_EINVAL, "out_host is NULL");
  const size_t bytes = ((size_t)1 << nq) * sizeof(uint64_t);
  uint64_t *d = nullptr;
  if (hipMalloc(&d, bytes) != hipSuccess) {
    (void)hipGetLastError();
    return fail(QCW_ENOMEM, "hipMalloc(%zu) failed", bytes);
  }
  rc = launch_pick(g, d, nullptr);
  if (!rc && hipMemcpy(out_host, d, bytes, hipMemcpyDeviceToHost) != hipSuccess)
    rc = fail(QCW_EHIP, "copy of labels failed");
  (void)hipFree(d);
  return rc;
}

int qcw_timing_enable(int on) {
  TimingState &t = ts();
  std::lock_guard<std::mutex> lk(t.mu);
  t.on = on != 0;
  return QCW_OK;
}

int qcw_timing_reset(void) {
  TimingState &t = ts();
  std::lock_guard<std::mutex> lk(t.mu);
  drain(t);
  for (int i = 0; i < QCW_KERNEL_COUNT; ++i) {
    t.launches[i] = 0;
    t.ms[i] = 0.0;
  }
  return QCW_OK;
}

int qcw_timing_read(int kernel, int64_t *launches, double *total_ms) {
  if (kernel < 0 || kernel >= QCW_KERNEL_COUNT || !launches || !total_ms)
    return fail(QCW_EINVAL, "bad timing query");
  TimingState &t = ts();
  std::lock_guard<std::mutex> lk(t.mu);
  drain(t);
  *launches = t.launches[kernel];
  *total_ms = t.ms[kernel];
  return QCW_OK;
}

}  // extern "C"

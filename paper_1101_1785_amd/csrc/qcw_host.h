// Host-side internals shared by the library's translation units: error state,
// argument validation, gate geometry and kernel timing.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

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
// Density matrices (multiverse step): rho of nq <= kRhoMaxQubits qubits is a
// 2nq-qubit vector.  launch_conjugate applies U rho U^dagger in one pass of
// 2^kConjTileBits-element LDS tiles (conjugate.hip), bit for bit the sweep of
// U on the row qubits followed by the sweep of conj(U) on the column qubits;
// targets validated by the caller, nq >= kConjTileBits / 2.
constexpr int kRhoMaxQubits = 17;
constexpr int kConjTileBits = 10;
int launch_conjugate(int nq, int k, const int *targets, const qcw_c64 *U, qcw_c64 *rho,
                     hipStream_t s);

// The plain circuit path for states of at most kSmallMaxQubits qubits: the
// whole (validated) circuit in one launch with the state in LDS, bit for bit
// one sweep per gate (small_circuit.hip).
constexpr int kSmallMaxQubits = 11;
int run_small_circuit(qcw_c64 *psi, int nq, const Geom *geo, const qcw_gate *gates, int ngates,
                      const qcw_c64 *mats, hipStream_t s);

int launch_sweep(const Geom &g, const qcw_c64 *U, const qcw_c64 *in, qcw_c64 *out,
                 hipStream_t s);
int launch_pick(const Geom &g, uint64_t *labels_dev, hipStream_t s);
// Fused passes (fused.hip).
// in_scratch: the plan tables go into the library's static per-GPU array
// (qcw_circuit_fused_noalloc) instead of a per-stream allocation.
int run_fused(qcw_c64 *psi, int nq, const qcw_gate *gates, int ngates, const qcw_c64 *mats,
              int tile_bits, int low_bits, int threads, int plan, hipStream_t s,
              bool in_scratch = false);
// Pass count of a plan; when non-NULL, pass_of[g] receives gate g's pass and
// order[] the gate indices in execution order.
int fused_pass_count(int nq, const qcw_gate *gates, int ngates, int tile_bits, int low_bits,
                     int plan, int *pass_of, int *order);
// Gate fusion (gate_fusion.cpp): gates idx[0..n) (all n gates when idx is
// NULL), in that order, merged greedily into blocks spanning at most
// max_qubits qubits, one gate per block; a gate joins a block only if the
// merged gate costs at most max_extra_flops more flops per amplitude than the
// block and the gate apart (8 * 2^k - 2 for k qubits).  Without regroup a
// block is a run of consecutive gates; with it, a gate may also join ahead of
// gates it shares no qubit with (they commute).  Output matrix offsets index
// *out_mats.  The gates must already be valid.
int fuse_gate_list(const qcw_gate *gates, const int *idx, int n, const qcw_c64 *mats,
                   int max_qubits, int max_extra_flops, bool regroup,
                   std::vector<qcw_gate> *out_gates, std::vector<qcw_c64> *out_mats);

}  // namespace qcw

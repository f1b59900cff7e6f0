// Internal types of the batched (persistent, LDS-resident) gate path.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "qcw_host.h"

namespace qcw {

constexpr int kBatchBlock = 256;     // at most 4 wavefronts, each on its own instance
constexpr int kBatchMaxNq = 12;      // largest instance kept in one wavefront's LDS
constexpr int kKernelBatch = 4;      // timing family of the batch kernel

// Tile-shape variants (see batch.hip).
enum BatchVariant : int32_t {
  kVarAmp4Sgpr = 0,
  kVarAmp8Sgpr = 1,
  kVarAmp16Sgpr = 2,
  kVarAmp4Lds = 3,
  kVarAmp8Lds = 4,
  kVarAmp4Mfma = 5,  // k = 2, 3 on FP64 matrix cores: equal to the plain path to rounding only
  kVarCount = 6
};
const char *variant_name(int v);
int variant_from_name(const char *s);

struct BInst {  // device copy of qcw_instance
  int32_t nq;
  int32_t ngates;
  int64_t state_off;
  int64_t gate_off;
};

struct alignas(16) BGate {  // gate with its geometry precomputed on the host
  int32_t k;
  int32_t sb0, sb1, sb2;    // target bits sorted ascending
  uint32_t off[8];          // member offsets, local index order
  int64_t mat_off;          // in complex elements
  int64_t pad;
};
static_assert(sizeof(BGate) == 64, "BGate layout");

// A work item carries its instance's fields and the first two gates'
// matrices, so a wave issues its state, descriptor and first operand loads
// at once.
struct alignas(16) BItem {
  int32_t nq;
  int32_t variant;    // BatchVariant
  int32_t g_begin;    // gate range of this launch (relative to gate_off)
  int32_t g_end;
  int64_t state_off;  // in complex elements
  int64_t gate_off;   // index of the instance's first gate
  int64_t mat0, mat1;  // matrix offsets of gates g_begin and g_begin + 1 (0: no such gate)
  int32_t k0, k1;      // their qubit counts
  int32_t pad[2];
};
static_assert(sizeof(BItem) == 64, "BItem layout");

// Grid of one of the two persistent kernels.
struct BatchShape {
  int wave_amps = 0;     // amplitudes of LDS state per wavefront
  size_t lds_bytes = 0;  // dynamic LDS per block
  int threads = 0;
  unsigned blocks = 0;
};

struct BatchLaunch {
  const BItem *items;  // items [0, n_exact) run in the exact kernel, the rest in
  int nitems;          // the matrix-core kernel (variant kVarAmp4Mfma)
  int n_exact;
  const BGate *gates;
  const double2 *mats;
  double2 *states;
  int *counter;        // two work counters: exact kernel, matrix-core kernel
  BatchShape ex, mf;
};

// Enqueues the reset of the work counters (when needed) and both kernels.
int launch_batch(const BatchLaunch &L, hipStream_t s);
int batch_kernel_occupancy(size_t lds_bytes, int threads, int *blocks_per_cu);
// The matrix-core kernel (batch_mfma.hip).
int launch_batch_mfma(const BatchLaunch &L, hipStream_t s);
int batch_mfma_occupancy(size_t lds_bytes, int threads, int *blocks_per_cu);

// Per-qubit-count variant choice, loaded from a tune table or the defaults.
struct TuneTable {
  int variant[kBatchMaxNq + 1];
  bool from_file = false;
};
void tune_defaults(TuneTable *t);
int tune_load(const char *path, TuneTable *t);

// Geometry of a gate for the batch kernel; validates like make_geom.
int make_bgate(int nq, const qcw_gate &g, int64_t nmats, BGate *out);

// Fuses gates spanning at most max_qubits qubits into one gate per block
// (gate_fusion.cpp): runs of consecutive gates, or with regroup also gates
// that commute past the ones between them; output matrix offsets index
// *out_mats.
int fuse_circuit(int nq, const qcw_gate *gates, int ngates, const qcw_c64 *mats, int64_t nmats,
                 int max_qubits, bool regroup, std::vector<qcw_gate> *out_gates,
                 std::vector<qcw_c64> *out_mats);

// Sizes both persistent kernels for n_exact and n_mfma items of at most
// max_nq qubits (a kernel with no items gets no grid).
int plan_batch_launch(int max_nq, int n_exact, int n_mfma, BatchLaunch *L);

}  // namespace qcw

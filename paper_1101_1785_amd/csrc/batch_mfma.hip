// Matrix-core form of the batched path (tile shape "amp4_mfma").
//
// Same work decomposition as the exact form (batch.hip): one wavefront per
// instance, the state resident in the wave's LDS for the whole circuit,
// written back once.  The circuits were fused on the host into gates of at
// most three qubits (gate_fusion.cpp).  Two- and three-qubit gates run on the
// FP64 matrix cores; one-qubit gates (rare after fusion) on the vector ALU.
// The summation order differs from the plain path, so results agree with it
// to rounding, not bit for bit.
//
// The gate updates themselves (real form of the complex product, lane
// layouts of the FP64 matrix-core instructions) are in mfma_gates.h.  Each
// lane's one or two matrix entries are prefetched from HBM into registers one
// gate ahead, so a wave keeps no copy of the matrix in LDS and its LDS holds
// the state alone.
#include <hip/hip_runtime.h>

#include "batch_common.h"
#include "mfma_gates.h"
#include "qcw_batch.h"
#include "qcw_device.h"

namespace qcw {

namespace {

__device__ void run_mfma_instance(const BInst &in, const BGate *__restrict__ gates,
                                  const double2 *__restrict__ mats, double2 *__restrict__ states,
                                  double2 *S, int lane, int g_begin, int g_end) {
  const int nq = in.nq;
  const uint32_t N = 1u << nq;
  double2 *st = states + in.state_off;
  load_state(S, st, N, lane);
  if (g_begin < g_end) {
    // Descriptors arrive two gates ahead, matrix operands one gate ahead.
    const uint32_t *gd = reinterpret_cast<const uint32_t *>(gates + in.gate_off);
    auto operands = [&](uint32_t d) {
      return mc::fetch_operands((int)desc_field(d, 0), mats + desc_mat(d), lane);
    };
    uint32_t dcur = load_desc(gd, g_begin, g_end, lane);
    uint32_t dnext = load_desc(gd, g_begin + 1, g_end, lane);
    mc::Operands nxt = operands(dcur);
    for (int gi = g_begin; gi < g_end; ++gi) {
      const mc::Fields f = mc::fields_of(dcur);
      const double2 u0 = nxt.p0, u1 = nxt.p1;
      const uint32_t dnext2 = load_desc(gd, gi + 2, g_end, lane);
      if (gi + 1 < g_end) nxt = operands(dnext);
      wave_lds_sync();
      mc::apply(S, 0, 1u << (nq - f.k), f, u0, u1, lane);
      dcur = dnext;
      dnext = dnext2;
    }
  }
  wave_lds_sync();
  store_state(S, st, N, lane);
}

// One persistent launch over the matrix-core items.  Each wavefront owns
// `wave_amps` amplitudes of dynamic LDS (no matrix slots).
__global__ __launch_bounds__(kBatchBlock) void batch_mfma_kernel(
    const BItem *__restrict__ items, int nitems, const BInst *__restrict__ inst,
    const BGate *__restrict__ gates, const double2 *__restrict__ mats,
    double2 *__restrict__ states, int *__restrict__ counter, int wave_amps) {
  extern __shared__ double2 lds[];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  double2 *S = lds + (size_t)wave * wave_amps;
  for_each_item(items, nitems, counter, lane, wave, [&](const BItem &item) {
    run_mfma_instance(inst[item.inst], gates, mats, states, S, lane, item.g_begin, item.g_end);
  });
}

}  // namespace

int launch_batch_mfma(const BatchLaunch &L, hipStream_t s) {
  const int n = L.nitems - L.n_exact;
  if (n <= 0) return QCW_OK;
  TimedLaunch t(kKernelBatch, s);
  hipLaunchKernelGGL(batch_mfma_kernel, dim3(L.mf.blocks), dim3(L.mf.threads), L.mf.lds_bytes, s,
                     L.items + L.n_exact, n, L.inst, L.gates, L.mats, L.states, L.counter + 1,
                     L.mf.wave_amps);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(QCW_EHIP, "matrix-core batch launch: %s", hipGetErrorString(e));
  return QCW_OK;
}

int batch_mfma_occupancy(size_t lds_bytes, int threads, int *blocks_per_cu) {
  int nb = 0;
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, batch_mfma_kernel, threads,
                                                              lds_bytes);
  if (e != hipSuccess) return fail(QCW_EHIP, "occupancy query: %s", hipGetErrorString(e));
  *blocks_per_cu = nb;
  return QCW_OK;
}

}  // namespace qcw

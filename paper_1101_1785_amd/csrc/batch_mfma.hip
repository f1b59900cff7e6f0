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

// Instances of at most kPreGates gates (after fusion: every circuit of up to
// ~40 random gates on 9 qubits) take all their gate descriptors into four
// registers at the start, beside the state load: register i, lane l holds
// dword l & 15 of gate 4 i + (l >> 4).  Each gate's matrix operands are then
// fetched two gates ahead into one of two register slots, taken in turn, so
// no register with a load in flight is ever copied.  Longer circuits stream
// their descriptors two gates ahead and operands one gate ahead.
constexpr int kPreGates = 16;

// A register copy the compiler cannot fold away: after it the slot's old
// value is dead, so the slot's refill can land in the same registers (left to
// itself the compiler feeds the gate straight from the slot and gives the
// refill new registers, which it then moves back behind a wait for the load).
__device__ __forceinline__ double2 copy_out(double2 v) {
  double2 r;
  asm volatile("v_mov_b64 %0, %1" : "=v"(r.x) : "v"(v.x));
  asm volatile("v_mov_b64 %0, %1" : "=v"(r.y) : "v"(v.y));
  return r;
}

__device__ __forceinline__ uint32_t pre_desc(const uint32_t (&dv)[4], int r) {
  const int i = r >> 2;  // wave-uniform
  return i == 0 ? dv[0] : i == 1 ? dv[1] : i == 2 ? dv[2] : dv[3];
}

// Fields of the gate whose descriptor occupies lanes b .. b + 15 of d.
__device__ __forceinline__ mc::Fields fields_at(uint32_t d, int b) {
  mc::Fields f;
  f.k = (int)__builtin_amdgcn_readlane(d, b + 0);
  f.sb0 = (int)__builtin_amdgcn_readlane(d, b + 1);
  f.sb1 = (int)__builtin_amdgcn_readlane(d, b + 2);
  f.sb2 = (int)__builtin_amdgcn_readlane(d, b + 3);
  f.off1 = __builtin_amdgcn_readlane(d, b + 5);
  f.off2 = __builtin_amdgcn_readlane(d, b + 6);
  f.off4 = __builtin_amdgcn_readlane(d, b + 8);
  return f;
}
__device__ __forceinline__ int64_t mat_at(uint32_t d, int b) {
  return (int64_t)(((uint64_t)__builtin_amdgcn_readlane(d, b + 13) << 32) |
                   __builtin_amdgcn_readlane(d, b + 12));
}

// Loads the descriptors of an instance of at most kPreGates gates (issued
// before the state load, so the two latencies overlap).
__device__ __forceinline__ void preload_desc(const BItem &in, const BGate *__restrict__ gates,
                                             int lane, uint32_t (&dv)[4]) {
  const int ng = in.g_end - in.g_begin;
  const uint32_t *gd = reinterpret_cast<const uint32_t *>(gates + in.gate_off);
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int g = in.g_begin + 4 * i + (lane >> 4);
    dv[i] = 0u;
    if (4 * i < ng && g < in.g_end)
      dv[i] = __builtin_nontemporal_load(gd + (size_t)g * 16 + (lane & 15));
  }
}

__device__ void run_mfma_preloaded(const BItem &in, const uint32_t (&dv)[4],
                                   const mc::Operands &first, const mc::Operands &second,
                                   const double2 *__restrict__ mats, double2 *S, int lane,
                                   uint32_t N) {
  const int ng = in.g_end - in.g_begin;
  auto operands = [&](int r) {
    const uint32_t d = pre_desc(dv, r);
    const int b = (r & 3) * 16;
    return mc::fetch_operands((int)__builtin_amdgcn_readlane(d, b), mats + mat_at(d, b), lane);
  };
  // Gate r of the instance, its operands taken out of `slot`, which is then
  // refilled with those of gate r + 2 (the last gate's again near the end: a
  // refill is never conditional, so each load lands in its slot's registers
  // and no wait is needed until two gates later).
  auto step = [&](int r, mc::Operands &slot) {
    const uint32_t d = pre_desc(dv, r);
    const mc::Fields f = fields_at(d, (r & 3) * 16);
    const double2 u0 = copy_out(slot.p0), u1 = copy_out(slot.p1);
    slot = operands(min(r + 2, ng - 1));
    wave_lds_sync();
    mc::apply(S, 0, N >> f.k, f, u0, u1, lane);
  };
  mc::Operands oa = first;
  mc::Operands ob = second;
  int r = 0;
  for (; r + 1 < ng; r += 2) {
    step(r, oa);
    step(r + 1, ob);
  }
  if (r < ng) step(r, oa);
}

__device__ void run_mfma_streamed(const BItem &in, const BGate *__restrict__ gates,
                                  const double2 *__restrict__ mats, double2 *S, int lane,
                                  uint32_t N) {
  const int g_begin = in.g_begin, g_end = in.g_end;
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
    mc::apply(S, 0, N >> f.k, f, u0, u1, lane);
    dcur = dnext;
    dnext = dnext2;
  }
}

__device__ void run_mfma_instance(const BItem &in, const BGate *__restrict__ gates,
                                  const double2 *__restrict__ mats, double2 *__restrict__ states,
                                  double2 *S, int lane) {
  const uint32_t N = 1u << in.nq;
  double2 *st = states + in.state_off;
  const int ng = in.g_end - in.g_begin;
  if (ng > 0 && ng <= kPreGates) {
    // the first two gates' operands come straight from the item, beside the
    // descriptor and state loads (one gate: the first gate's again)
    const mc::Operands first = mc::fetch_operands(in.k0, mats + in.mat0, lane);
    const mc::Operands second = ng > 1 ? mc::fetch_operands(in.k1, mats + in.mat1, lane) : first;
    uint32_t dv[4];
    preload_desc(in, gates, lane, dv);
    load_state(S, st, N, lane);
    run_mfma_preloaded(in, dv, first, second, mats, S, lane, N);
  } else {
    load_state(S, st, N, lane);
    if (ng > 0) run_mfma_streamed(in, gates, mats, S, lane, N);
  }
  wave_lds_sync();
  store_state(S, st, N, lane);
}

// One persistent launch over the matrix-core items.  Each wavefront owns
// `wave_amps` amplitudes of dynamic LDS (no matrix slots).
__global__ __launch_bounds__(kBatchBlock) __attribute__((amdgpu_waves_per_eu(4))) void batch_mfma_kernel(
    const BItem *__restrict__ items, int nitems, const BGate *__restrict__ gates,
    const double2 *__restrict__ mats, double2 *__restrict__ states, int *__restrict__ counter,
    int wave_amps) {
  extern __shared__ double2 lds[];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  double2 *S = lds + (size_t)wave * wave_amps;
  for_each_item(items, nitems, counter, lane, wave, [&](const BItem &item) {
    run_mfma_instance(item, gates, mats, states, S, lane);
  });
}

}  // namespace

int launch_batch_mfma(const BatchLaunch &L, hipStream_t s) {
  const int n = L.nitems - L.n_exact;
  if (n <= 0) return QCW_OK;
  TimedLaunch t(kKernelBatch, s);
  hipLaunchKernelGGL(batch_mfma_kernel, dim3(L.mf.blocks), dim3(L.mf.threads), L.mf.lds_bytes, s,
                     L.items + L.n_exact, n, L.gates, L.mats, L.states, L.counter + 1,
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

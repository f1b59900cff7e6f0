// Batched form: many independent (state, circuit) instances in one persistent
// launch -- the paper's independent multiverse paths (§5), or independent
// requests.  Each wavefront takes instances (the host orders them largest
// first; waves beyond their first item pull from an atomic counter), copies the instance's state into its own
// LDS region once, applies every gate of its circuit there (Op1/Op2/Op3 of
// §3a-§3c, the same group arithmetic as the one-gate sweep), and writes the
// state back once.  HBM traffic per instance is therefore 32 * 2^nq bytes for
// the state plus its gate matrices, instead of 32 * 2^nq per gate.
//
// Tile shape per instance (chosen per qubit count by the autotuner):
//   amp     amplitudes each lane loads before computing (4, 8 or 16; 4 or 8
//           with a staged matrix), i.e. max(1, amp / 2^k) groups per lane
//   mat     where the wave reads the gate matrix: the scalar cache (wave-
//           uniform loads) or a copy staged in the wave's LDS.
// These shapes run the plain path's group arithmetic in its FMA order, so
// results equal the plain path bit for bit.  The matrix-core shape has its
// own kernel (batch_mfma.hip).
#include <hip/hip_runtime.h>

#include "batch_common.h"
#include "qcw_batch.h"
#include "qcw_device.h"

namespace qcw {

template <int K, int AMP, bool MAT_LDS>
__device__ __forceinline__ void lds_gate(double2 *S, int nq, const BGate &g, const double2 *U,
                                         const double2 *Ul, int lane) {
  constexpr int M = 1 << K;
  constexpr int ILP = AMP > M ? AMP / M : 1;
  // With the matrix staged in LDS, one-qubit gates copy it into registers once
  // (four broadcast reads) and reuse it for every group of the lane; larger
  // matrices are read from LDS per use (caching them costs occupancy).
  constexpr bool UREG = MAT_LDS && K == 1;
  double2 ureg[UREG ? M * M : 1];
  if (UREG) {
#pragma unroll
    for (int e = 0; e < M * M; ++e) ureg[UREG ? e : 0] = Ul[e];
  }
  const uint32_t ngroups = 1u << (nq - K);
  // insert_zeros deposits the bits of j into the non-target positions, so for
  // j = 64 m + lane it is the OR of the deposits of 64 m (wave-uniform) and of
  // lane (once per gate).
  const uint32_t lane_base = insert_zeros<K, uint32_t>((uint32_t)lane, g.sb0, g.sb1, g.sb2);
  for (uint32_t j0 = lane; j0 < ngroups; j0 += 64 * ILP) {
    double2 x[ILP][M];
    uint32_t base[ILP];
#pragma unroll
    for (int i = 0; i < ILP; ++i) {
      const uint32_t j = j0 + 64 * i;
      base[i] = lane_base | insert_zeros<K, uint32_t>(j0 - lane + 64 * i, g.sb0, g.sb1, g.sb2);
      if (j < ngroups) {
#pragma unroll
        for (int r = 0; r < M; ++r) x[i][r] = S[base[i] + g.off[r]];
      }
    }
#pragma unroll
    for (int i = 0; i < ILP; ++i) {
      const uint32_t j = j0 + 64 * i;
      if (j < ngroups) {
        const uint32_t b = base[i];
        auto put = [&](int r, double2 y) { S[b + g.off[r]] = y; };
        if (UREG)
          group_matvec_put<M>(x[i], [&](int r, int c) { return ureg[UREG ? r * M + c : 0]; }, put);
        else if (MAT_LDS)
          group_matvec_put<M>(x[i], [&](int r, int c) { return Ul[r * M + c]; }, put);
        else
          group_matvec_put<M>(x[i], [&](int r, int c) { return U[r * M + c]; }, put);
      }
    }
  }
}

template <int AMP, bool MAT_LDS>
__device__ void run_instance(const BItem &in, const BGate *__restrict__ gates,
                             const double2 *__restrict__ mats, double2 *__restrict__ states,
                             double2 *S, double2 *Ul, int lane, int g_begin, int g_end) {
  const int nq = in.nq;
  const uint32_t N = 1u << nq;
  double2 *st = states + in.state_off;
  load_state(S, st, N, lane);
  if (g_begin >= g_end) {
    wave_lds_sync();
    return;
  }
  // Descriptors arrive two gates ahead (load_desc).  The next gate's matrix
  // is fetched while the current gate runs (lane e holds entry e in flight)
  // and staged into one of two LDS slots.
  const uint32_t *gd = reinterpret_cast<const uint32_t *>(gates + in.gate_off);
  auto field = [](uint32_t d, int i) -> uint32_t { return desc_field(d, i); };
  auto mat_of = [](uint32_t d) -> int64_t { return desc_mat(d); };
  uint32_t dcur = load_desc(gd, g_begin, g_end, lane);
  uint32_t dnext = load_desc(gd, g_begin + 1, g_end, lane);
  double2 mreg = make_double2(0.0, 0.0);
  {
    const int k0 = (int)field(dcur, 0);
    if (MAT_LDS && lane < (1 << (2 * k0))) mreg = mats[mat_of(dcur) + lane];
  }
  for (int gi = g_begin; gi < g_end; ++gi) {
    BGate g;
    g.k = (int)field(dcur, 0);
    g.sb0 = (int)field(dcur, 1);
    g.sb1 = (int)field(dcur, 2);
    g.sb2 = (int)field(dcur, 3);
#pragma unroll
    for (int r = 0; r < 8; ++r) g.off[r] = field(dcur, 4 + r);
    g.mat_off = mat_of(dcur);
    double2 *Ub = Ul + ((gi - g_begin) & 1) * 64;
    if (MAT_LDS && lane < (1 << (2 * g.k))) Ub[lane] = mreg;
    wave_lds_sync();
    const double2 *U = mats + g.mat_off;
    const uint32_t dnext2 = load_desc(gd, gi + 2, g_end, lane);
    if (gi + 1 < g_end) {
      const int nk = (int)field(dnext, 0);
      if (MAT_LDS && lane < (1 << (2 * nk))) mreg = mats[mat_of(dnext) + lane];
    }
    switch (g.k) {
      case 1: lds_gate<1, AMP, MAT_LDS>(S, nq, g, U, Ub, lane); break;
      case 2: lds_gate<2, AMP, MAT_LDS>(S, nq, g, U, Ub, lane); break;
      default: lds_gate<3, AMP, MAT_LDS>(S, nq, g, U, Ub, lane); break;
    }
    dcur = dnext;
    dnext = dnext2;
  }
  wave_lds_sync();
  store_state(S, st, N, lane);
}

// One persistent launch over `nitems` work items.  Each wavefront owns
// `wave_amps` amplitudes of dynamic LDS plus two 64-entry matrix slots.
__global__ __launch_bounds__(kBatchBlock) void batch_kernel(
    const BItem *__restrict__ items, int nitems, const BGate *__restrict__ gates,
    const double2 *__restrict__ mats, double2 *__restrict__ states, int *__restrict__ counter,
    int wave_amps) {
  extern __shared__ double2 lds[];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  double2 *S = lds + (size_t)wave * (wave_amps + 128);
  double2 *Ul = S + wave_amps;
  for_each_item(items, nitems, counter, lane, wave, [&](const BItem &item) {
    const BItem &in = item;
    const int g0 = item.g_begin, g1 = item.g_end;
    switch (item.variant) {
      case kVarAmp4Sgpr: run_instance<4, false>(in, gates, mats, states, S, Ul, lane, g0, g1); break;
      case kVarAmp8Sgpr: run_instance<8, false>(in, gates, mats, states, S, Ul, lane, g0, g1); break;
      case kVarAmp16Sgpr: run_instance<16, false>(in, gates, mats, states, S, Ul, lane, g0, g1); break;
      case kVarAmp4Lds: run_instance<4, true>(in, gates, mats, states, S, Ul, lane, g0, g1); break;
      default: run_instance<8, true>(in, gates, mats, states, S, Ul, lane, g0, g1); break;
    }
  });
}

__global__ void reset_counter_kernel(int *counter) {
  if (threadIdx.x < 2 && blockIdx.x == 0) counter[threadIdx.x] = 0;
}

int launch_batch(const BatchLaunch &L, hipStream_t s) {
  const int n_mfma = L.nitems - L.n_exact;
  if (L.nitems == 0) return QCW_OK;
  hipError_t e;
  // A work counter is read only when a kernel's items outnumber its waves.
  const bool count_ex = L.n_exact > 0 && (int64_t)L.n_exact > (int64_t)L.ex.blocks * (L.ex.threads / 64);
  const bool count_mf = n_mfma > 0 && (int64_t)n_mfma > (int64_t)L.mf.blocks * (L.mf.threads / 64);
  if (count_ex || count_mf) {
    hipLaunchKernelGGL(reset_counter_kernel, dim3(1), dim3(64), 0, s, L.counter);
    e = hipGetLastError();
    if (e != hipSuccess) return fail(QCW_EHIP, "counter reset launch: %s", hipGetErrorString(e));
  }
  if (L.n_exact > 0) {
    TimedLaunch t(kKernelBatch, s);
    hipLaunchKernelGGL(batch_kernel, dim3(L.ex.blocks), dim3(L.ex.threads), L.ex.lds_bytes, s,
                       L.items, L.n_exact, L.gates, L.mats, L.states, L.counter,
                       L.ex.wave_amps);
    e = hipGetLastError();
    if (e != hipSuccess) return fail(QCW_EHIP, "batch launch: %s", hipGetErrorString(e));
  }
  if (n_mfma > 0) return launch_batch_mfma(L, s);
  return QCW_OK;
}

int batch_kernel_occupancy(size_t lds_bytes, int threads, int *blocks_per_cu) {
  int nb = 0;
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, batch_kernel, threads,
                                                              lds_bytes);
  if (e != hipSuccess) return fail(QCW_EHIP, "occupancy query: %s", hipGetErrorString(e));
  *blocks_per_cu = nb;
  return QCW_OK;
}

}  // namespace qcw

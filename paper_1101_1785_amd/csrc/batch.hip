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
#include <hip/hip_runtime.h>

#include "qcw_batch.h"
#include "qcw_device.h"

namespace qcw {

// Orders LDS traffic between the lanes of one wavefront: every LDS access of
// the wave issued before this point completes before any issued after it.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

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
  for (uint32_t j0 = lane; j0 < ngroups; j0 += 64 * ILP) {
    double2 x[ILP][M];
    uint32_t base[ILP];
#pragma unroll
    for (int i = 0; i < ILP; ++i) {
      const uint32_t j = j0 + 64 * i;
      base[i] = insert_zeros<K, uint32_t>(j, g.sb0, g.sb1, g.sb2);
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

// Copies an instance's 2^nq amplitudes from HBM into the wave's LDS region,
// eight loads in flight per lane before any LDS store when 2^nq >= 512.
__device__ __forceinline__ void load_state(double2 *S, const double2 *st, uint32_t N, int lane) {
  uint32_t n0 = 0;
  for (; n0 + 512 <= N; n0 += 512) {
    double2 v0 = st[n0 + lane], v1 = st[n0 + 64 + lane], v2 = st[n0 + 128 + lane],
            v3 = st[n0 + 192 + lane], v4 = st[n0 + 256 + lane], v5 = st[n0 + 320 + lane],
            v6 = st[n0 + 384 + lane], v7 = st[n0 + 448 + lane];
    S[n0 + lane] = v0;
    S[n0 + 64 + lane] = v1;
    S[n0 + 128 + lane] = v2;
    S[n0 + 192 + lane] = v3;
    S[n0 + 256 + lane] = v4;
    S[n0 + 320 + lane] = v5;
    S[n0 + 384 + lane] = v6;
    S[n0 + 448 + lane] = v7;
  }
  for (uint32_t n = n0 + lane; n < N; n += 64) S[n] = st[n];
}

template <int AMP, bool MAT_LDS>
__device__ void run_instance(const BInst &in, const BGate *__restrict__ gates,
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
  // The next gate's matrix is fetched while the current gate runs (lane e
  // holds entry e in flight) and staged into one of two LDS slots; reading the
  // next descriptor's k and matrix offset also brings its cache line in.
  int nk = gates[in.gate_off + g_begin].k;
  int64_t nmat = gates[in.gate_off + g_begin].mat_off;
  double2 mreg = make_double2(0.0, 0.0);
  if (MAT_LDS && lane < (1 << (2 * nk))) mreg = mats[nmat + lane];
  for (int gi = g_begin; gi < g_end; ++gi) {
    double2 *Ub = Ul + ((gi - g_begin) & 1) * 64;
    if (MAT_LDS && lane < (1 << (2 * nk))) Ub[lane] = mreg;
    wave_lds_sync();
    const BGate g = gates[in.gate_off + gi];
    const double2 *U = mats + g.mat_off;
    if (gi + 1 < g_end) {
      nk = gates[in.gate_off + gi + 1].k;
      nmat = gates[in.gate_off + gi + 1].mat_off;
      if (MAT_LDS && lane < (1 << (2 * nk))) mreg = mats[nmat + lane];
    }
    switch (g.k) {
      case 1: lds_gate<1, AMP, MAT_LDS>(S, nq, g, U, Ub, lane); break;
      case 2: lds_gate<2, AMP, MAT_LDS>(S, nq, g, U, Ub, lane); break;
      default: lds_gate<3, AMP, MAT_LDS>(S, nq, g, U, Ub, lane); break;
    }
  }
  wave_lds_sync();
  for (uint32_t n = lane; n < N; n += 64) st[n] = S[n];
}

// One persistent launch over `nitems` work items.  Each wavefront owns
// `wave_amps` amplitudes of dynamic LDS plus two 64-entry matrix slots.
__global__ __launch_bounds__(kBatchBlock) void batch_kernel(
    const BItem *__restrict__ items, int nitems, const BInst *__restrict__ inst,
    const BGate *__restrict__ gates, const double2 *__restrict__ mats,
    double2 *__restrict__ states, int *__restrict__ counter, int wave_amps) {
  extern __shared__ double2 lds[];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  double2 *S = lds + (size_t)wave * (wave_amps + 128);
  double2 *Ul = S + wave_amps;
  // The first item of every wave is static (items are ordered largest first);
  // only when items outnumber waves do waves pull more from the counter, so a
  // batch that fits the grid takes no atomics at all.
  const int waves_per_block = blockDim.x >> 6;
  const int total_waves = gridDim.x * waves_per_block;
  // wave-uniform by construction; readfirstlane lets the compiler keep the
  // item, instance and gate data in scalar registers
  int it = __builtin_amdgcn_readfirstlane(blockIdx.x * waves_per_block + wave);
  while (it < nitems) {
    const BItem item = items[it];
    const BInst in = inst[item.inst];
    const int g0 = item.g_begin, g1 = item.g_end;
    switch (item.variant) {
      case kVarAmp4Sgpr: run_instance<4, false>(in, gates, mats, states, S, Ul, lane, g0, g1); break;
      case kVarAmp8Sgpr: run_instance<8, false>(in, gates, mats, states, S, Ul, lane, g0, g1); break;
      case kVarAmp16Sgpr: run_instance<16, false>(in, gates, mats, states, S, Ul, lane, g0, g1); break;
      case kVarAmp4Lds: run_instance<4, true>(in, gates, mats, states, S, Ul, lane, g0, g1); break;
      default: run_instance<8, true>(in, gates, mats, states, S, Ul, lane, g0, g1); break;
    }
    // The LDS region is reused by the next item only after this wave's
    // stores of the current one were issued (wave order); no other wave uses it.
    wave_lds_sync();
    if (nitems <= total_waves) break;
    int nx = 0;
    if (lane == 0) nx = atomicAdd(counter, 1);
    it = total_waves + __builtin_amdgcn_readfirstlane(__shfl(nx, 0));
  }
}

__global__ void reset_counter_kernel(int *counter) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *counter = 0;
}

int launch_batch(const BatchLaunch &L, hipStream_t s) {
  hipLaunchKernelGGL(reset_counter_kernel, dim3(1), dim3(64), 0, s, L.counter);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(QCW_EHIP, "counter reset launch: %s", hipGetErrorString(e));
  if (L.nitems == 0) return QCW_OK;
  TimedLaunch t(kKernelBatch, s);
  hipLaunchKernelGGL(batch_kernel, dim3(L.blocks), dim3(L.threads), L.lds_bytes, s, L.items,
                     L.nitems, L.inst, L.gates, L.mats, L.states, L.counter, L.wave_amps);
  e = hipGetLastError();
  if (e != hipSuccess) return fail(QCW_EHIP, "batch launch: %s", hipGetErrorString(e));
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

// Device helpers shared by the two persistent batch kernels (batch.hip, the
// exact form, and batch_mfma.hip, the matrix-core form).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "qcw_batch.h"

namespace qcw {

// Orders LDS traffic between the lanes of one wavefront.  A wavefront's LDS
// instructions are executed in issue order, so a read issued after a write by
// another lane of the same wave sees it; only the compiler must not move LDS
// accesses across this point.  (No other wave touches the region.)
__device__ __forceinline__ void wave_lds_sync() { __asm__ volatile("" ::: "memory"); }

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
  if (n0 == 0) {
    // 2^nq <= 256 (at most four amplitudes per lane): every load issued
    // before any LDS store, in named registers (an array here went to scratch)
    const uint32_t a = lane, b = 64 + lane, c = 128 + lane, d = 192 + lane;
    double2 va = make_double2(0.0, 0.0), vb = va, vc = va, vd = va;
    if (a < N) va = st[a];
    if (b < N) vb = st[b];
    if (c < N) vc = st[c];
    if (d < N) vd = st[d];
    if (a < N) S[a] = va;
    if (b < N) S[b] = vb;
    if (c < N) S[c] = vc;
    if (d < N) S[d] = vd;
    return;
  }
  for (uint32_t n = n0 + lane; n < N; n += 64) S[n] = st[n];
}

__device__ __forceinline__ void store_state(const double2 *S, double2 *st, uint32_t N, int lane) {
  for (uint32_t n = lane; n < N; n += 64) st[n] = S[n];
}

// Gate descriptors travel through vector loads: lane d < 16 holds dword d of
// a 64-byte BGate (k, sb0..sb2, off[0..7], mat_off), and fields are read with
// readlane.  No scalar load (whose wait would also drain the LDS queue) then
// sits between gates.
__device__ __forceinline__ uint32_t load_desc(const uint32_t *gd, int gi, int g_end, int lane) {
  return (gi < g_end && lane < 16) ? __builtin_nontemporal_load(gd + (size_t)gi * 16 + lane) : 0u;
}
__device__ __forceinline__ uint32_t desc_field(uint32_t d, int i) {
  return __builtin_amdgcn_readlane(d, i);
}
__device__ __forceinline__ int64_t desc_mat(uint32_t d) {
  return (int64_t)(((uint64_t)desc_field(d, 13) << 32) | desc_field(d, 12));
}

// The item loop of a persistent kernel: the first item of every wave is
// static (items are ordered largest first); only when items outnumber waves
// do waves pull more from the counter, so a batch that fits the grid takes no
// atomics at all.  The item index is wave-uniform by construction;
// readfirstlane lets the compiler keep item and instance data in scalar
// registers.
template <typename Run>
__device__ __forceinline__ void for_each_item(const BItem *__restrict__ items, int nitems,
                                              int *__restrict__ counter, int lane, int wave,
                                              Run run) {
  const int waves_per_block = blockDim.x >> 6;
  const int total_waves = gridDim.x * waves_per_block;
  int it = __builtin_amdgcn_readfirstlane(blockIdx.x * waves_per_block + wave);
  while (it < nitems) {
    run(items[it]);
    // The LDS region is reused by the next item only after this wave's
    // accesses to the current one were issued (wave order).
    wave_lds_sync();
    if (nitems <= total_waves) break;
    int nx = 0;
    if (lane == 0) nx = atomicAdd(counter, 1);
    it = total_waves + __builtin_amdgcn_readfirstlane(__shfl(nx, 0));
  }
}

}  // namespace qcw

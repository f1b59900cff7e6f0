// rho <- U rho U^dagger in one pass over rho (the algorithm gates of the
// multiverse step, Eq. rhoE4).  Read as a vector, rho is a 2nq-qubit state;
// U acts on the row qubits and conj(U) on the column qubits.  Instead of one
// sweep for each, a block takes a tile of 2^kConjTileBits elements closed
// under both gates' target bits and the four lowest bits (so a tile is made
// of contiguous 16-element chunks), applies U then conj(U) inside the tile in
// LDS, and writes the tile back: one read and one write of rho.  Each gate is
// the sweep's group update (members in the same order, the same products in
// the same order), so the result equals the two sweeps bit for bit.
#include <hip/hip_runtime.h>

#include <string.h>

#include <algorithm>

#include "qcw_device.h"
#include "qcw_host.h"

namespace qcw {

namespace {

constexpr int kConjThreads = 256;
constexpr int kConjLow = 4;  // label bits 0..3 are always tile bits

template <int K>
struct ConjArgs {
  uint32_t tile_pos[kConjTileBits];    // label bits of the tile, ascending (the first kConjLow are 0..3)
  uint32_t outer_pos[2 * kRhoMaxQubits];  // the other label bits, ascending
  int32_t nouter;
  int32_t sb_r[3], sb_c[3];            // local (tile-index) target bits, ascending
  uint32_t off_r[1 << K], off_c[1 << K];  // local member offsets, local index order
  double2 u[(1 << K) * (1 << K)];      // U, row-major
  double2 uc[(1 << K) * (1 << K)];     // conj(U)
};

template <int K>
__device__ __forceinline__ void conj_gate(double2 *S, const int (&sb)[3], const uint32_t (&off)[1 << K],
                                          const double2 *u) {
  constexpr int M = 1 << K;
  constexpr uint32_t NG = 1u << (kConjTileBits - K);
  for (uint32_t j = threadIdx.x; j < NG; j += kConjThreads) {
    const uint32_t base = insert_zeros<K, uint32_t>(j, sb[0], sb[1], sb[2]);
    double2 x[M];
#pragma unroll
    for (int r = 0; r < M; ++r) x[r] = S[base + off[r]];
    double2 y[M];
    group_matvec<M>(x, y, [&](int r, int c) { return u[r * M + c]; });
#pragma unroll
    for (int r = 0; r < M; ++r) S[base + off[r]] = y[r];
  }
}

template <int K>
__global__ __launch_bounds__(kConjThreads) void conj_tile_kernel(double2 *rho, ConjArgs<K> a) {
  constexpr int N_TILE = 1 << kConjTileBits;
  constexpr int PER = N_TILE / kConjThreads;
  __shared__ double2 S[N_TILE];
  __shared__ uint64_t chunk[N_TILE >> kConjLow];  // label offset of each 16-element chunk
  uint64_t base = 0;
  {
    const uint64_t b = blockIdx.x;
    for (int j = 0; j < a.nouter; ++j) base |= ((b >> j) & 1ull) << a.outer_pos[j];
  }
  for (uint32_t c = threadIdx.x; c < (N_TILE >> kConjLow); c += kConjThreads) {
    uint64_t o = 0;
#pragma unroll
    for (int j = 0; j < kConjTileBits - kConjLow; ++j)
      o |= (uint64_t)((c >> j) & 1u) << a.tile_pos[kConjLow + j];
    chunk[c] = base | o;
  }
  __syncthreads();
  uint64_t lab[PER];
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const uint32_t i = q * kConjThreads + threadIdx.x;
    lab[q] = chunk[i >> kConjLow] | (i & ((1u << kConjLow) - 1));
    S[i] = rho[lab[q]];
  }
  __syncthreads();
  conj_gate<K>(S, a.sb_r, a.off_r, a.u);
  __syncthreads();
  conj_gate<K>(S, a.sb_c, a.off_c, a.uc);
  __syncthreads();
#pragma unroll
  for (int q = 0; q < PER; ++q) rho[lab[q]] = S[q * kConjThreads + threadIdx.x];
}

template <int K>
int launch_k(int nq, const int *targets, const qcw_c64 *U, qcw_c64 *rho, hipStream_t s) {
  const int nb = 2 * nq;  // label bits of the superket
  ConjArgs<K> a;
  memset(&a, 0, sizeof(a));
  // Target bits: row qubit t is label bit nb - t, column qubit t is bit nq - t.
  int rbit[3], cbit[3];
  uint64_t mask = (1ull << kConjLow) - 1;
  for (int j = 0; j < K; ++j) {
    rbit[j] = nb - targets[j];
    cbit[j] = nq - targets[j];
    mask |= (1ull << rbit[j]) | (1ull << cbit[j]);
  }
  // widen with the lowest unused bits to kConjTileBits tile bits
  for (int b = 0; b < nb && __builtin_popcountll(mask) < kConjTileBits; ++b) mask |= 1ull << b;
  int nt = 0, no = 0, local[64];
  for (int b = 0; b < nb; ++b) {
    if ((mask >> b) & 1) {
      local[b] = nt;
      a.tile_pos[nt++] = (uint32_t)b;
    } else {
      a.outer_pos[no++] = (uint32_t)b;
    }
  }
  a.nouter = no;
  auto geom = [&](const int (&bits)[3], int32_t (&sb)[3], uint32_t (&off)[1 << K]) {
    int sorted[3] = {0, 0, 0};
    for (int j = 0; j < K; ++j) sorted[j] = local[bits[j]];
    std::sort(sorted, sorted + K);
    for (int j = 0; j < 3; ++j) sb[j] = sorted[j];
    // member r: the first listed target is the most significant bit of r
    for (int r = 0; r < (1 << K); ++r) {
      uint32_t o = 0;
      for (int j = 0; j < K; ++j)
        if ((r >> (K - 1 - j)) & 1) o |= 1u << local[bits[j]];
      off[r] = o;
    }
  };
  geom(rbit, a.sb_r, a.off_r);
  geom(cbit, a.sb_c, a.off_c);
  for (int i = 0; i < (1 << K) * (1 << K); ++i) {
    a.u[i] = make_double2(U[i].re, U[i].im);
    a.uc[i] = make_double2(U[i].re, -U[i].im);
  }
  const uint64_t blocks = 1ull << (nb - kConjTileBits);
  if (blocks > 0x7fffffffull) return fail(QCW_EINVAL, "rho too large for one launch");
  TimedLaunch t(QCW_KERNEL_CONJ, s);
  hipLaunchKernelGGL(conj_tile_kernel<K>, dim3((unsigned)blocks), dim3(kConjThreads), 0, s,
                     reinterpret_cast<double2 *>(rho), a);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(QCW_EHIP, "conjugation launch: %s", hipGetErrorString(e));
  return QCW_OK;
}

}  // namespace

int launch_conjugate(int nq, int k, const int *targets, const qcw_c64 *U, qcw_c64 *rho,
                     hipStream_t s) {
  switch (k) {
    case 1: return launch_k<1>(nq, targets, U, rho, s);
    case 2: return launch_k<2>(nq, targets, U, rho, s);
    case 3: return launch_k<3>(nq, targets, U, rho, s);
  }
  return fail(QCW_EINVAL, "k must be 1, 2 or 3");
}

}  // namespace qcw

// One-gate sweep: QCWAVE's Op1 / Op2 / Op3 (§3a-§3c) on a state in HBM.
// (Gates on the two lowest qubits and others among the lowest 12 run as
// contiguous LDS tiles instead: sweep_low_kernel below.)
//
// Each thread takes GPT groups (pairs, quartets or octets).  Group j's base
// label comes from inserting zero bits at the sorted target positions; member
// r adds off[r] (the strides of the targets whose value in r is 1).  Consecutive
// lanes take consecutive j, so for every member the wavefront's 64 loads cover
// contiguous 16-byte amplitudes whenever the lowest target bit is >= 6, and
// whole cache lines across the members otherwise.  All loads of a thread are
// issued before any arithmetic, so a thread keeps GPT * m loads in flight, and
// each amplitude is read once and written once: 32 bytes of HBM traffic per
// amplitude per gate.  The m x m matrix travels in the kernel arguments and is
// read through the scalar cache (wave-uniform), never from a per-lane load.
#include <hip/hip_runtime.h>

#include "qcw_device.h"
#include "qcw_host.h"

namespace qcw {

typedef double v2d __attribute__((ext_vector_type(2)));

template <bool NT>
__device__ __forceinline__ double2 ld2(const double2 *p) {
  v2d v;
  if (NT)
    v = __builtin_nontemporal_load(reinterpret_cast<const v2d *>(p));
  else
    v = *reinterpret_cast<const v2d *>(p);
  return make_double2(v.x, v.y);
}

template <bool NT>
__device__ __forceinline__ void st2(double2 *p, double2 a) {
  v2d v = {a.x, a.y};
  if (NT)
    __builtin_nontemporal_store(v, reinterpret_cast<v2d *>(p));
  else
    *reinterpret_cast<v2d *>(p) = v;
}

template <int K>
struct MatArg {
  double2 u[(1 << K) * (1 << K)];
};

template <typename I>
struct SweepArg {
  I ngroups;
  I off[8];
  int sb0, sb1, sb2;
};

constexpr int kSweepBlock = 256;

template <int K, int GPT, typename I, bool NT>
__global__ __launch_bounds__(kSweepBlock) void sweep_kernel(const double2 *in, double2 *out,
                                                            SweepArg<I> a, MatArg<K> U) {
  constexpr int M = 1 << K;
  double2 x[GPT][M];
  I base[GPT];
  const I j0 = (I)blockIdx.x * (I)(GPT * kSweepBlock) + (I)threadIdx.x;
#pragma unroll
  for (int i = 0; i < GPT; ++i) {
    const I j = j0 + (I)(i * kSweepBlock);
    base[i] = insert_zeros<K, I>(j, a.sb0, a.sb1, a.sb2);
    if (j < a.ngroups) {
#pragma unroll
      for (int r = 0; r < M; ++r) x[i][r] = ld2<NT>(in + (base[i] + a.off[r]));
    }
  }
#pragma unroll
  for (int i = 0; i < GPT; ++i) {
    const I j = j0 + (I)(i * kSweepBlock);
    if (j < a.ngroups) {
      double2 y[M];
      group_matvec<M>(x[i], y, [&](int r, int c) { return U.u[r * M + c]; });
#pragma unroll
      for (int r = 0; r < M; ++r) st2<NT>(out + (base[i] + a.off[r]), y[r]);
    }
  }
}

// Pick_k labels as the sweep computes them (test support).
template <int K>
__global__ void pick_kernel(uint64_t *labels, SweepArg<uint64_t> a) {
  constexpr int M = 1 << K;
  const uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= a.ngroups) return;
  const uint64_t base = insert_zeros<K, uint64_t>(j, a.sb0, a.sb1, a.sb2);
#pragma unroll
  for (int r = 0; r < M; ++r) labels[j * M + r] = base + a.off[r];
}

template <typename I>
static SweepArg<I> sweep_arg(const Geom &g) {
  SweepArg<I> a{};
  a.ngroups = (I)((uint64_t)1 << (g.nq - g.k));
  for (int r = 0; r < (1 << g.k); ++r) a.off[r] = (I)g.off[r];
  a.sb0 = g.sb[0];
  a.sb1 = g.sb[1];
  a.sb2 = g.sb[2];
  return a;
}

template <int K, int GPT, typename I>
static int launch_k(const Geom &g, const qcw_c64 *U, const qcw_c64 *in, qcw_c64 *out,
                    hipStream_t s) {
  MatArg<K> m;
  for (int i = 0; i < (1 << K) * (1 << K); ++i) m.u[i] = make_double2(U[i].re, U[i].im);
  SweepArg<I> a = sweep_arg<I>(g);
  const uint64_t per_block = (uint64_t)GPT * kSweepBlock;
  const uint64_t blocks = ((uint64_t)a.ngroups + per_block - 1) / per_block;
  if (blocks > 0x7fffffffULL) return fail(QCW_EINVAL, "state too large for one launch");
  TimedLaunch t(K, s);
  hipLaunchKernelGGL((sweep_kernel<K, GPT, I, false>), dim3((unsigned)blocks), dim3(kSweepBlock),
                     0, s, reinterpret_cast<const double2 *>(in),
                     reinterpret_cast<double2 *>(out), a, m);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(QCW_EHIP, "sweep launch: %s", hipGetErrorString(e));
  return QCW_OK;
}

// Gates whose targets all lie in the lowest kLowTileBits label bits and
// include bits 0 and 1: a group's members then form runs of 4 or 8 adjacent
// amplitudes, and in sweep_kernel each member load of a wavefront touches a
// separate cache line per lane.  Here each block instead moves one contiguous
// tile of 2^kLowTileBits amplitudes through LDS with coalesced loads and
// stores, and applies the gate to the tile's groups there, with the same
// products in the same order as sweep_kernel (so the same bits).
constexpr int kLowTileBits = 12;
constexpr int kLowBlock = 512;

template <int K>
__global__ __launch_bounds__(kLowBlock) void sweep_low_kernel(const double2 *in, double2 *out,
                                                              SweepArg<uint32_t> a, MatArg<K> U) {
  constexpr int M = 1 << K;
  constexpr int TILE = 1 << kLowTileBits;
  constexpr int PER = TILE / kLowBlock;
  constexpr int G = (TILE / M) / kLowBlock;  // groups per thread
  extern __shared__ double2 S[];
  const uint64_t t0 = (uint64_t)blockIdx.x << kLowTileBits;
  v2d v[PER];
#pragma unroll
  for (int q = 0; q < PER; ++q)
    v[q] = *reinterpret_cast<const v2d *>(in + t0 + q * kLowBlock + threadIdx.x);
#pragma unroll
  for (int q = 0; q < PER; ++q) S[q * kLowBlock + threadIdx.x] = make_double2(v[q].x, v[q].y);
  __syncthreads();
  double2 x[G][M];
  uint32_t base[G];
#pragma unroll
  for (int i = 0; i < G; ++i) {
    base[i] = insert_zeros<K, uint32_t>(i * kLowBlock + threadIdx.x, a.sb0, a.sb1, a.sb2);
#pragma unroll
    for (int r = 0; r < M; ++r) x[i][r] = S[base[i] + a.off[r]];
  }
#pragma unroll
  for (int i = 0; i < G; ++i) {
    double2 y[M];
    group_matvec<M>(x[i], y, [&](int r, int c) { return U.u[r * M + c]; });
#pragma unroll
    for (int r = 0; r < M; ++r) S[base[i] + a.off[r]] = y[r];
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const double2 y = S[q * kLowBlock + threadIdx.x];
    *reinterpret_cast<v2d *>(out + t0 + q * kLowBlock + threadIdx.x) = v2d{y.x, y.y};
  }
}

template <int K>
static int launch_low(const Geom &g, const qcw_c64 *U, const qcw_c64 *in, qcw_c64 *out,
                      hipStream_t s) {
  MatArg<K> m;
  for (int i = 0; i < (1 << K) * (1 << K); ++i) m.u[i] = make_double2(U[i].re, U[i].im);
  SweepArg<uint32_t> a = sweep_arg<uint32_t>(g);
  const uint64_t blocks = (uint64_t)1 << (g.nq - kLowTileBits);
  if (blocks > 0x7fffffffULL) return fail(QCW_EINVAL, "state too large for one launch");
  const size_t lds = sizeof(double2) << kLowTileBits;
  TimedLaunch t(K, s);
  hipLaunchKernelGGL((sweep_low_kernel<K>), dim3((unsigned)blocks), dim3(kLowBlock), lds, s,
                     reinterpret_cast<const double2 *>(in), reinterpret_cast<double2 *>(out), a, m);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(QCW_EHIP, "sweep launch: %s", hipGetErrorString(e));
  return QCW_OK;
}

int launch_sweep(const Geom &g, const qcw_c64 *U, const qcw_c64 *in, qcw_c64 *out,
                 hipStream_t s) {
  // Targets within the lowest tile bits, including bits 0 and 1: LDS tiles.
  if (g.k >= 2 && g.nq >= kLowTileBits && g.nq <= 31 && g.sb[0] == 0 && g.sb[1] == 1 &&
      g.sb[g.k - 1] < kLowTileBits)
    return g.k == 2 ? launch_low<2>(g, U, in, out, s) : launch_low<3>(g, U, in, out, s);
  // 32-bit labels while every label and shift fits (nq <= 31), 64-bit above.
  const bool small = g.nq <= 31;
  switch (g.k) {
    case 1:
      return small ? launch_k<1, 4, uint32_t>(g, U, in, out, s)
                   : launch_k<1, 4, uint64_t>(g, U, in, out, s);
    case 2:
      return small ? launch_k<2, 2, uint32_t>(g, U, in, out, s)
                   : launch_k<2, 2, uint64_t>(g, U, in, out, s);
    case 3:
      return small ? launch_k<3, 1, uint32_t>(g, U, in, out, s)
                   : launch_k<3, 1, uint64_t>(g, U, in, out, s);
  }
  return fail(QCW_EINVAL, "k must be 1, 2 or 3");
}

int launch_pick(const Geom &g, uint64_t *labels_dev, hipStream_t s) {
  SweepArg<uint64_t> a = sweep_arg<uint64_t>(g);
  const unsigned blocks = (unsigned)((a.ngroups + 255) / 256);
  switch (g.k) {
    case 1: hipLaunchKernelGGL(pick_kernel<1>, dim3(blocks), dim3(256), 0, s, labels_dev, a); break;
    case 2: hipLaunchKernelGGL(pick_kernel<2>, dim3(blocks), dim3(256), 0, s, labels_dev, a); break;
    case 3: hipLaunchKernelGGL(pick_kernel<3>, dim3(blocks), dim3(256), 0, s, labels_dev, a); break;
    default: return fail(QCW_EINVAL, "k must be 1, 2 or 3");
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(QCW_EHIP, "pick launch: %s", hipGetErrorString(e));
  return QCW_OK;
}

}  // namespace qcw

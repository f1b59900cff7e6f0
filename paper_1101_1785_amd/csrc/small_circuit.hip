// The plain circuit path on states small enough for one block's LDS
// (nq <= 11, 32 KiB): the whole circuit in one launch instead of one sweep
// launch per gate.  The state is loaded into LDS once; each gate is the
// one-gate sweep's group update (Op1 / Op2 / Op3 of §3a-§3c: groups from
// inserting zeros at the sorted target bits, members in the sweep's order, the
// same products in the same order), with a block barrier between gates; the
// state is stored back at the end.  So the result equals one sweep per gate
// bit for bit.  Gates and their matrices travel in the kernel arguments and
// are copied into LDS at the start; a circuit that does not fit one argument
// block runs as several launches, in order.
#include <hip/hip_runtime.h>

#include "qcw_device.h"
#include "qcw_host.h"

namespace qcw {

namespace {

constexpr int kSmallBlock = 256;
constexpr int kSmallGates = 32;   // gates per launch
constexpr int kSmallMats = 224;   // complex matrix entries per launch

struct SmallGate {
  uint8_t k;
  uint8_t sb[3];    // target bits, ascending
  uint8_t bit[3];   // target bits, argument order (the first is the MSB of r)
  uint8_t pad;
  uint16_t mat;     // first entry of its m x m matrix in SmallArgs::m
  uint16_t pad2;
};
static_assert(sizeof(SmallGate) == 12, "SmallGate layout");
static_assert(sizeof(double2) << kSmallMaxQubits <= 32 * 1024, "state and arguments fit 64 KiB of LDS");

struct alignas(16) SmallArgs {  // 3984 bytes: with the state pointer, within one argument block
  int32_t nq, ngates;
  SmallGate g[kSmallGates];
  double2 m[kSmallMats];
};

template <int K>
__device__ __forceinline__ void small_gate(double2 *S, int nq, const SmallGate &g,
                                           const double2 *m) {
  constexpr int M = 1 << K;
  uint32_t off[M];
#pragma unroll
  for (int r = 0; r < M; ++r) {
    uint32_t o = 0;
#pragma unroll
    for (int j = 0; j < K; ++j)
      if ((r >> (K - 1 - j)) & 1) o |= 1u << g.bit[j];
    off[r] = o;
  }
  const uint32_t ng = 1u << (nq - K);
  for (uint32_t j = threadIdx.x; j < ng; j += kSmallBlock) {
    const uint32_t base = insert_zeros<K, uint32_t>(j, g.sb[0], g.sb[1], g.sb[2]);
    double2 x[M];
#pragma unroll
    for (int r = 0; r < M; ++r) x[r] = S[base + off[r]];
    group_matvec_put<M>(x, [&](int r, int c) { return m[g.mat + r * M + c]; },
                        [&](int r, double2 y) { S[base + off[r]] = y; });
  }
}

// The argument block is copied into LDS once, by all threads together: read
// from its own segment gate by gate, each gate would wait for a separate
// round trip to it.
__global__ __launch_bounds__(kSmallBlock) void small_circuit_kernel(double2 *psi, SmallArgs A) {
  __shared__ double2 S[1 << kSmallMaxQubits];
  __shared__ SmallArgs C;
  {
    const uint4 *src = reinterpret_cast<const uint4 *>(&A);
    uint4 *dst = reinterpret_cast<uint4 *>(&C);
    for (uint32_t i = threadIdx.x; i < sizeof(SmallArgs) / sizeof(uint4); i += kSmallBlock)
      dst[i] = src[i];
  }
  const int nq = A.nq, ngates = A.ngates;
  const uint32_t n = 1u << nq;
  for (uint32_t i = threadIdx.x; i < n; i += kSmallBlock) S[i] = psi[i];
  __syncthreads();
  for (int gi = 0; gi < ngates; ++gi) {
    const SmallGate g = C.g[gi];
    switch (g.k) {
      case 1: small_gate<1>(S, nq, g, C.m); break;
      case 2: small_gate<2>(S, nq, g, C.m); break;
      default: small_gate<3>(S, nq, g, C.m); break;
    }
    __syncthreads();
  }
  for (uint32_t i = threadIdx.x; i < n; i += kSmallBlock) psi[i] = S[i];
}

int launch_small(qcw_c64 *psi, const SmallArgs &a, hipStream_t s) {
  TimedLaunch t(QCW_KERNEL_SMALL, s);
  hipLaunchKernelGGL(small_circuit_kernel, dim3(1), dim3(kSmallBlock), 0, s,
                     reinterpret_cast<double2 *>(psi), a);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(QCW_EHIP, "small circuit launch: %s", hipGetErrorString(e));
  return QCW_OK;
}

}  // namespace

int run_small_circuit(qcw_c64 *psi, int nq, const Geom *geo, const qcw_gate *gates, int ngates,
                      const qcw_c64 *mats, hipStream_t s) {
  if (nq < 1 || nq > kSmallMaxQubits) return fail(QCW_EINVAL, "nq=%d outside [1, %d]", nq, kSmallMaxQubits);
  SmallArgs a;
  a.nq = nq;
  a.ngates = 0;
  int nm = 0;
  for (int i = 0; i < ngates; ++i) {
    const Geom &g = geo[i];
    const int mm = 1 << (2 * g.k);
    if (a.ngates == kSmallGates || nm + mm > kSmallMats) {  // this launch is full
      const int rc = launch_small(psi, a, s);
      if (rc) return rc;
      a.ngates = 0;
      nm = 0;
    }
    SmallGate &d = a.g[a.ngates++];
    d = SmallGate{};
    d.k = (uint8_t)g.k;
    for (int j = 0; j < 3; ++j) {
      d.sb[j] = (uint8_t)g.sb[j];
      d.bit[j] = (uint8_t)g.bit[j];
    }
    d.mat = (uint16_t)nm;
    const qcw_c64 *U = mats + gates[i].mat;
    for (int e = 0; e < mm; ++e) a.m[nm + e] = make_double2(U[e].re, U[e].im);
    nm += mm;
  }
  return a.ngates > 0 ? launch_small(psi, a, s) : QCW_OK;
}

}  // namespace qcw

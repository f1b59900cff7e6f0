// Device-side building blocks shared by every kernel of the library, so that
// the one-gate sweep, the batched kernel and the fused passes perform the same
// floating-point operations in the same order for every group (their results
// are bit-identical to one another).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace qcw {

// acc + u * x with four fused multiply-adds in a fixed order.
__device__ __forceinline__ double2 cmad(double2 acc, double2 u, double2 x) {
  acc.x = __fma_rn(u.x, x.x, acc.x);
  acc.x = __fma_rn(-u.y, x.y, acc.x);
  acc.y = __fma_rn(u.x, x.y, acc.y);
  acc.y = __fma_rn(u.y, x.x, acc.y);
  return acc;
}

// y[r] = sum_c U[r][c] x[c] for one group (§3a Eq. resmat1, §3b Eq. resmat2),
// c ascending, accumulator starting at +0.  U is read through `u(r, c)`.
template <int M, typename MatFn>
__device__ __forceinline__ void group_matvec(const double2 (&x)[M], double2 (&y)[M],
                                             MatFn u) {
#pragma unroll
  for (int r = 0; r < M; ++r) {
    double2 acc = make_double2(0.0, 0.0);
#pragma unroll
    for (int c = 0; c < M; ++c) acc = cmad(acc, u(r, c), x[c]);
    y[r] = acc;
  }
}

// The same products as group_matvec, each output row handed to `put(r, y_r)`
// as soon as it is complete (fewer live registers; inputs must already be
// loaded, which makes in-place updates safe).
template <int M, typename MatFn, typename PutFn>
__device__ __forceinline__ void group_matvec_put(const double2 (&x)[M], MatFn u, PutFn put) {
#pragma unroll
  for (int r = 0; r < M; ++r) {
    double2 acc = make_double2(0.0, 0.0);
#pragma unroll
    for (int c = 0; c < M; ++c) acc = cmad(acc, u(r, c), x[c]);
    put(r, acc);
  }
}

// Group index j -> lowest label of its group: a zero bit is inserted at each
// target bit position, taken in ascending order (sb0 < sb1 < sb2).
template <int K, typename I>
__device__ __forceinline__ I insert_zeros(I j, int sb0, int sb1, int sb2) {
  I x = j;
  x = ((x >> sb0) << (sb0 + 1)) | (x & ((I(1) << sb0) - I(1)));
  if (K >= 2) x = ((x >> sb1) << (sb1 + 1)) | (x & ((I(1) << sb1) - I(1)));
  if (K >= 3) x = ((x >> sb2) << (sb2 + 1)) | (x & ((I(1) << sb2) - I(1)));
  return x;
}

}  // namespace qcw

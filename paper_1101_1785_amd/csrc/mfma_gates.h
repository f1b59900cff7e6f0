// Gate updates on an LDS-resident block of amplitudes with the FP64 matrix
// cores, for the matrix-core batch kernel (batch_mfma.hip).  A wavefront
// applies a gate to a range of its groups; the results agree with the plain
// path to rounding (the instructions' summation order), not bit for bit.
//
// The complex m x m product is the real 2m x 2m product
//   [Re y; Im y] = [[Re U, -Im U], [Im U, Re U]] [Re x; Im x]
// over many groups at once (one group per column).  Lane layouts of the two
// instructions used (l = lane), read off the hardware with an in-bounds probe:
//   v_mfma_f64_4x4x4f64, four independent 4x4x4 blocks, block (l >> 2) & 3:
//     A[l & 3][l >> 4], B[l >> 4][l & 3], D[l >> 4][l & 3]
//   v_mfma_f64_16x16x4f64:
//     A[l & 15][l >> 4], B[l >> 4][l & 15], D[4v + (l >> 4)][l & 15], v = 0..3
// Each lane holds only the one or two matrix entries its A operand needs, and
// reads and writes back exactly the amplitudes it owns, so a gate needs no
// exchange between the lanes of a wave.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "qcw_device.h"

namespace qcw {
namespace mc {

typedef double d4 __attribute__((ext_vector_type(4)));

// At most this many tiles of 16 groups are applied together by one step:
// their LDS latencies and matrix-core chains overlap.  A gate with fewer
// groups (small instances: 2^(nq-k) groups) issues only the tiles it has.
constexpr int kTiles = 4;

// Gate descriptor header (the first twelve dwords of both BGate and
// FusedGate): k, sb0..sb2 (target bits, ascending), off[0..7] (member
// offsets in local index order).  A wave holds it lane-distributed (lane d <
// 16 holds dword d) and reads fields with readlane.
struct Fields {
  int k, sb0, sb1, sb2;
  uint32_t off1, off2, off4;  // strides of local bits 0, 1, 2 (off[1 << j])
};

__device__ __forceinline__ Fields fields_of(uint32_t d) {
  Fields f;
  f.k = (int)__builtin_amdgcn_readlane(d, 0);
  f.sb0 = (int)__builtin_amdgcn_readlane(d, 1);
  f.sb1 = (int)__builtin_amdgcn_readlane(d, 2);
  f.sb2 = (int)__builtin_amdgcn_readlane(d, 3);
  f.off1 = __builtin_amdgcn_readlane(d, 5);
  f.off2 = __builtin_amdgcn_readlane(d, 6);
  f.off4 = __builtin_amdgcn_readlane(d, 8);
  return f;
}

// Offset of local index r from its group's base (first target = most
// significant bit of r).
__device__ __forceinline__ uint32_t member(const Fields &f, int r) {
  return ((r & 1) ? f.off1 : 0u) + ((r & 2) ? f.off2 : 0u) + ((r & 4) ? f.off4 : 0u);
}

// The matrix entries lane `lane` needs for a k-qubit gate with matrix U
// (row-major):
//   k = 3: U[r][s] and U[r][4 + s], r = 4 ((l & 15) >> 3) + (l & 3), s = l >> 4
//   k = 2: U[l & 3][l >> 4]
//   k = 1: U[l & 3] (lanes 0..3 hold the whole 2 x 2 matrix)
// Both loads are always issued (for k < 3 the second repeats the first), so
// the operands stay in registers.
struct Operands {
  double2 p0, p1;
};
__device__ __forceinline__ Operands fetch_operands(int k, const double2 *__restrict__ U, int lane) {
  const int row = lane & 15, r = 4 * (row >> 3) + (row & 3), s = lane >> 4;
  const int i0 = k == 3 ? r * 8 + s : (k == 2 ? (lane & 3) * 4 + s : (lane & 3));
  const int i1 = k == 3 ? r * 8 + 4 + s : i0;
  Operands o;
  o.p0 = U[i0];
  o.p1 = U[i1];
  return o;
}

__device__ __forceinline__ double lane_double(double v, int l) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
  return __hiloint2double(hi, lo);
}

// Group ranges: the wave applies the gate to groups jb .. jb + nj - 1 of the
// block.  jb is a multiple of 64 (or 0).  Group bases are zero-bit
// insertions (bit deposits), so the base of group jb + t0 + 16 t + (l & 15)
// is the OR of the deposit of the wave-uniform part and of l & 15.

// One-qubit gate on the vector ALU: the 2 x 2 matrix is made wave-uniform
// (readlane from lanes 0..3); each lane takes four groups per step.
__device__ __forceinline__ void gate1(double2 *S, uint32_t jb, uint32_t nj, const Fields &f,
                                      double2 p0, int lane) {
  double2 u[4];
#pragma unroll
  for (int e = 0; e < 4; ++e) u[e] = make_double2(lane_double(p0.x, e), lane_double(p0.y, e));
  const uint32_t lane_base = insert_zeros<1, uint32_t>((uint32_t)lane, f.sb0, 0, 0);
  for (uint32_t j0 = 0; j0 < nj; j0 += 256) {
    double2 x0[4], x1[4];
    uint32_t b[4];
    bool ok[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      ok[t] = j0 + 64 * t + lane < nj;
      b[t] = lane_base | insert_zeros<1, uint32_t>(jb + j0 + 64 * t, f.sb0, 0, 0);
      if (ok[t]) {
        x0[t] = S[b[t]];
        x1[t] = S[b[t] + f.off1];
      }
    }
#pragma unroll
    for (int t = 0; t < 4; ++t)
      if (ok[t]) {
        double2 y0 = make_double2(0.0, 0.0), y1 = y0;
        y0 = cmad(y0, u[0], x0[t]);
        y0 = cmad(y0, u[1], x1[t]);
        y1 = cmad(y1, u[2], x0[t]);
        y1 = cmad(y1, u[3], x1[t]);
        S[b[t]] = y0;
        S[b[t] + f.off1] = y1;
      }
  }
}

// Two-qubit gate, 16 groups per tile: the real 8 x 8 matrix splits into four
// 4 x 4 blocks acting on (Re x, Im x):
//   Re y = ReU Re x - ImU Im x,  Im y = ImU Re x + ReU Im x.
// Lane l holds U[l & 3][l >> 4] and owns amplitude l >> 4 of its group.  NT
// tiles per step; FULL: nj is a multiple of 16 NT, so no tile needs masking.
template <int NT, bool FULL>
__device__ __forceinline__ void gate2(double2 *S, uint32_t jb, uint32_t nj, const Fields &f,
                                      double2 u, int lane) {
  const uint32_t lane_p =
      insert_zeros<2, uint32_t>((uint32_t)(lane & 15), f.sb0, f.sb1, 0) + member(f, lane >> 4);
  const bool lane_ok = FULL || (uint32_t)(lane & 15) < nj;
  for (uint32_t t0 = 0; t0 < nj; t0 += 16 * NT) {
    uint32_t p[NT];
    bool ok[NT];
    double2 x[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      ok[t] = FULL || (lane_ok && t0 + 16 * t < nj);
      p[t] = lane_p | insert_zeros<2, uint32_t>(jb + t0 + 16 * t, f.sb0, f.sb1, 0);
      x[t] = make_double2(0.0, 0.0);
      if (ok[t]) x[t] = S[p[t]];
    }
    double re[NT], im[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      re[t] = __builtin_amdgcn_mfma_f64_4x4x4f64(u.x, x[t].x, 0.0, 0, 0, 0);
      im[t] = __builtin_amdgcn_mfma_f64_4x4x4f64(u.y, x[t].x, 0.0, 0, 0, 0);
    }
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      re[t] = __builtin_amdgcn_mfma_f64_4x4x4f64(-u.y, x[t].y, re[t], 0, 0, 0);
      im[t] = __builtin_amdgcn_mfma_f64_4x4x4f64(u.x, x[t].y, im[t], 0, 0, 0);
    }
#pragma unroll
    for (int t = 0; t < NT; ++t)
      if (ok[t]) S[p[t]] = make_double2(re[t], im[t]);
  }
}

// Three-qubit gate, 16 groups per tile.  Real index of (amplitude c, part p)
// is 8 (c >> 2) + 4 p + (c & 3), so a lane's four output rows (4v + (l >> 4))
// are Re, Im of amplitude s = l >> 4 and Re, Im of amplitude 4 + s -- the two
// amplitudes it also supplies as B.  Lane l holds the A entries of its row
// l & 15 (fetch_operands): real parts for a Re row, and the signs and parts
// of the real form for an Im row.  NT tiles per step, FULL as for gate2.
template <int NT, bool FULL>
__device__ __forceinline__ void gate3(double2 *S, uint32_t jb, uint32_t nj, const Fields &f,
                                      double2 u0, double2 u1, int lane) {
  const int s = lane >> 4;
  const bool im_row = (lane >> 2) & 1;
  const double a0 = im_row ? u0.y : u0.x, a1 = im_row ? u0.x : -u0.y;
  const double a2 = im_row ? u1.y : u1.x, a3 = im_row ? u1.x : -u1.y;
  const uint32_t m0 = member(f, s), m1 = member(f, 4 + s);
  const uint32_t lane_b = insert_zeros<3, uint32_t>((uint32_t)(lane & 15), f.sb0, f.sb1, f.sb2);
  const bool lane_ok = FULL || (uint32_t)(lane & 15) < nj;
  for (uint32_t t0 = 0; t0 < nj; t0 += 16 * NT) {
    uint32_t b[NT];
    bool ok[NT];
    double2 x0[NT], x1[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      ok[t] = FULL || (lane_ok && t0 + 16 * t < nj);
      b[t] = lane_b | insert_zeros<3, uint32_t>(jb + t0 + 16 * t, f.sb0, f.sb1, f.sb2);
      x0[t] = make_double2(0.0, 0.0);
      x1[t] = x0[t];
      if (ok[t]) {
        x0[t] = S[b[t] + m0];
        x1[t] = S[b[t] + m1];
      }
    }
    d4 d[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      d[t] = d4{0.0, 0.0, 0.0, 0.0};
      d[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, x0[t].x, d[t], 0, 0, 0);
    }
#pragma unroll
    for (int t = 0; t < NT; ++t) d[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, x0[t].y, d[t], 0, 0, 0);
#pragma unroll
    for (int t = 0; t < NT; ++t) d[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a2, x1[t].x, d[t], 0, 0, 0);
#pragma unroll
    for (int t = 0; t < NT; ++t) d[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a3, x1[t].y, d[t], 0, 0, 0);
#pragma unroll
    for (int t = 0; t < NT; ++t)
      if (ok[t]) {
        S[b[t] + m0] = make_double2(d[t][0], d[t][1]);
        S[b[t] + m1] = make_double2(d[t][2], d[t][3]);
      }
  }
}

// One gate of descriptor f with operands (u0, u1) on groups jb .. jb + nj - 1
// (nj a power of two): as many tiles per step as there are groups, up to
// kTiles.  Each group's result depends only on its own column, so the tile
// count changes no result.
__device__ __forceinline__ void apply(double2 *S, uint32_t jb, uint32_t nj, const Fields &f,
                                      double2 u0, double2 u1, int lane) {
  if (f.k == 3) {
    if (nj >= 16 * kTiles) gate3<kTiles, true>(S, jb, nj, f, u0, u1, lane);
    else if (nj == 32) gate3<2, true>(S, jb, nj, f, u0, u1, lane);
    else if (nj == 16) gate3<1, true>(S, jb, nj, f, u0, u1, lane);
    else gate3<1, false>(S, jb, nj, f, u0, u1, lane);
  } else if (f.k == 2) {
    if (nj >= 16 * kTiles) gate2<kTiles, true>(S, jb, nj, f, u0, lane);
    else if (nj == 32) gate2<2, true>(S, jb, nj, f, u0, lane);
    else if (nj == 16) gate2<1, true>(S, jb, nj, f, u0, lane);
    else gate2<1, false>(S, jb, nj, f, u0, lane);
  } else {
    gate1(S, jb, nj, f, u0, lane);
  }
}

}  // namespace mc
}  // namespace qcw

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
//   mfma    two- and three-qubit gates on the FP64 matrix cores (below); the
//           summation order differs from the plain path, so results agree with
//           it to rounding rather than bit for bit.
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

// ---- FP64 matrix-core gates ------------------------------------------------
// The complex m x m product is the real 2m x 2m product
//   [Re y; Im y] = [[Re U, -Im U], [Im U, Re U]] [Re x; Im x]
// over many groups at once (one group per column).  Lane layouts of the two
// instructions used (l = lane):
//   v_mfma_f64_4x4x4f64, four independent 4x4x4 blocks, block (l >> 2) & 3:
//     A[l & 3][l >> 4], B[l >> 4][l & 3], D[l >> 4][l & 3]
//   v_mfma_f64_16x16x4f64:
//     A[l & 15][l >> 4], B[l >> 4][l & 15], D[4v + (l >> 4)][l & 15], v = 0..3
// The matrix is spread over the lanes (each lane holds one or two entries), so
// no lane needs the whole matrix; every lane reads and writes back exactly the
// amplitudes it owns, so a gate needs no exchange between lanes.
typedef double qcw_d4 __attribute__((ext_vector_type(4)));

// Offset of local index r from its group's base: the first target is the most
// significant bit of r, and off[1 << j] is the stride of local bit j.
template <int K>
__device__ __forceinline__ uint32_t member_off(const BGate &g, int r) {
  uint32_t o = (r & 1) ? g.off[1] : 0u;
  if (K >= 2 && (r & 2)) o += g.off[2];
  if (K >= 3 && (r & 4)) o += g.off[4];
  return o;
}

// Two-qubit gate, 16 groups per step: columns are groups t0 + (l & 15); the
// real 8 x 8 matrix splits into four 4 x 4 blocks acting on (Re x, Im x):
//   Re y = ReU Re x - ImU Im x,  Im y = ImU Re x + ReU Im x.
// Lane l holds U[l & 3][l >> 4] and owns amplitude l >> 4 of its group.
__device__ __forceinline__ void mfma_gate2(double2 *S, int nq, const BGate &g, const double2 *Ul,
                                           int lane) {
  const uint32_t ngroups = 1u << (nq - 2);
  const int r = lane >> 4;
  const double2 u = Ul[(lane & 3) * 4 + r];
  const uint32_t moff = member_off<2>(g, r);
  for (uint32_t t0 = 0; t0 < ngroups; t0 += 32) {
    const uint32_t ja = t0 + (lane & 15), jb = ja + 16;
    const bool oka = ja < ngroups, okb = jb < ngroups;
    const uint32_t pa = insert_zeros<2, uint32_t>(ja, g.sb0, g.sb1, g.sb2) + moff;
    const uint32_t pb = insert_zeros<2, uint32_t>(jb, g.sb0, g.sb1, g.sb2) + moff;
    double2 xa = make_double2(0.0, 0.0), xb = make_double2(0.0, 0.0);
    if (oka) xa = S[pa];
    if (okb) xb = S[pb];
    double ra = __builtin_amdgcn_mfma_f64_4x4x4f64(u.x, xa.x, 0.0, 0, 0, 0);
    double ia = __builtin_amdgcn_mfma_f64_4x4x4f64(u.y, xa.x, 0.0, 0, 0, 0);
    double rb = __builtin_amdgcn_mfma_f64_4x4x4f64(u.x, xb.x, 0.0, 0, 0, 0);
    double ib = __builtin_amdgcn_mfma_f64_4x4x4f64(u.y, xb.x, 0.0, 0, 0, 0);
    ra = __builtin_amdgcn_mfma_f64_4x4x4f64(-u.y, xa.y, ra, 0, 0, 0);
    ia = __builtin_amdgcn_mfma_f64_4x4x4f64(u.x, xa.y, ia, 0, 0, 0);
    rb = __builtin_amdgcn_mfma_f64_4x4x4f64(-u.y, xb.y, rb, 0, 0, 0);
    ib = __builtin_amdgcn_mfma_f64_4x4x4f64(u.x, xb.y, ib, 0, 0, 0);
    if (oka) S[pa] = make_double2(ra, ia);
    if (okb) S[pb] = make_double2(rb, ib);
  }
}

// Three-qubit gate, 16 groups per step.  Real index of (amplitude c, part p)
// is 8 (c >> 2) + 4 p + (c & 3), so a lane's four output rows (4v + (l >> 4))
// are Re, Im of amplitude s = l >> 4 and Re, Im of amplitude 4 + s -- the two
// amplitudes it also supplies as B.  Lane l holds the A entries of row
// l & 15: U[r][s] and U[r][4 + s] with r = 4 ((l & 15) >> 3) + (l & 3).
__device__ __forceinline__ void mfma_gate3(double2 *S, int nq, const BGate &g, const double2 *Ul,
                                           int lane) {
  const uint32_t ngroups = 1u << (nq - 3);
  const int s = lane >> 4, row = lane & 15;
  const int r = 4 * (row >> 3) + (row & 3);
  const bool im_row = (row >> 2) & 1;
  const double2 u0 = Ul[r * 8 + s], u1 = Ul[r * 8 + 4 + s];
  const double a0 = im_row ? u0.y : u0.x, a1 = im_row ? u0.x : -u0.y;
  const double a2 = im_row ? u1.y : u1.x, a3 = im_row ? u1.x : -u1.y;
  const uint32_t m0 = member_off<3>(g, s), m1 = member_off<3>(g, 4 + s);
  for (uint32_t t0 = 0; t0 < ngroups; t0 += 32) {
    const uint32_t ja = t0 + (lane & 15), jb = ja + 16;
    const bool oka = ja < ngroups, okb = jb < ngroups;
    const uint32_t ba = insert_zeros<3, uint32_t>(ja, g.sb0, g.sb1, g.sb2);
    const uint32_t bb = insert_zeros<3, uint32_t>(jb, g.sb0, g.sb1, g.sb2);
    double2 xa0 = make_double2(0.0, 0.0), xa1 = xa0, xb0 = xa0, xb1 = xa0;
    if (oka) {
      xa0 = S[ba + m0];
      xa1 = S[ba + m1];
    }
    if (okb) {
      xb0 = S[bb + m0];
      xb1 = S[bb + m1];
    }
    qcw_d4 da = {0.0, 0.0, 0.0, 0.0}, db = {0.0, 0.0, 0.0, 0.0};
    da = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, xa0.x, da, 0, 0, 0);
    db = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, xb0.x, db, 0, 0, 0);
    da = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, xa0.y, da, 0, 0, 0);
    db = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, xb0.y, db, 0, 0, 0);
    da = __builtin_amdgcn_mfma_f64_16x16x4f64(a2, xa1.x, da, 0, 0, 0);
    db = __builtin_amdgcn_mfma_f64_16x16x4f64(a2, xb1.x, db, 0, 0, 0);
    da = __builtin_amdgcn_mfma_f64_16x16x4f64(a3, xa1.y, da, 0, 0, 0);
    db = __builtin_amdgcn_mfma_f64_16x16x4f64(a3, xb1.y, db, 0, 0, 0);
    if (oka) {
      S[ba + m0] = make_double2(da[0], da[1]);
      S[ba + m1] = make_double2(da[2], da[3]);
    }
    if (okb) {
      S[bb + m0] = make_double2(db[0], db[1]);
      S[bb + m1] = make_double2(db[2], db[3]);
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

template <int AMP, bool MAT_LDS, bool MFMA = false>
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
      case 2:
        if (MFMA) mfma_gate2(S, nq, g, Ub, lane);
        else lds_gate<2, AMP, MAT_LDS>(S, nq, g, U, Ub, lane);
        break;
      default:
        if (MFMA) mfma_gate3(S, nq, g, Ub, lane);
        else lds_gate<3, AMP, MAT_LDS>(S, nq, g, U, Ub, lane);
        break;
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
      case kVarAmp4Mfma: run_instance<4, true, true>(in, gates, mats, states, S, Ul, lane, g0, g1); break;
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
  if (L.nitems == 0) return QCW_OK;
  hipError_t e;
  // The work counter is read only when items outnumber the grid's waves.
  if ((int64_t)L.nitems > (int64_t)L.blocks * (L.threads / 64)) {
    hipLaunchKernelGGL(reset_counter_kernel, dim3(1), dim3(64), 0, s, L.counter);
    e = hipGetLastError();
    if (e != hipSuccess) return fail(QCW_EHIP, "counter reset launch: %s", hipGetErrorString(e));
  }
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

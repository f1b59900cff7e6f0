// One GPU's part of a gate on a state split over two GPUs by its top qubit.
//
// The paper's MPI predecessor distributes the state vector over processors
// (§5, general remarks; §1).  With qubit 1 the most significant bit of the
// label (§2c, Eq. staten), splitting by qubit 1 gives each of two GPUs one
// contiguous half: rank d holds the 2^(nq-1) amplitudes whose qubit 1 equals
// d.  A gate whose targets avoid qubit 1 is the one-gate sweep on each half.
// A gate on qubit 1 (and up to two local qubits) needs the partner's half:
// after an exchange (on MI355X an xGMI transfer; not part of this library),
// each rank forms every group from its own members and the partner's staged
// members and writes only its own rows.  The group arithmetic is the sweep's
// (same member order, same FMA sequence), so the two halves together equal
// qcw_opk on the whole state bit for bit.
//
// Traffic per local amplitude: 16 B of the own half read + written, 16 B of
// the staged half read: 48 B.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "qcw_device.h"
#include "qcw_host.h"

namespace qcw {

namespace {

constexpr int kShardBlock = 256;

template <int K>
struct ShardArg {
  double2 u[(1 << K) * (1 << K)];  // full gate matrix, row-major
  uint64_t ngroups;                // local groups: 2^(nq - 1 - (K - 1))
  uint64_t loff[1 << K];           // local offset of member r
  int sb0, sb1;                    // local target bits, ascending (K - 1 of them)
  int gshift;                      // member r lies in the global half (r >> gshift) & 1
  int rank;                        // this share's value of qubit 1
};

template <int K>
__global__ __launch_bounds__(kShardBlock) void shard_kernel(double2 *__restrict__ loc,
                                                            const double2 *__restrict__ rem,
                                                            ShardArg<K> a) {
  constexpr int M = 1 << K;
  const uint64_t j = (uint64_t)blockIdx.x * kShardBlock + threadIdx.x;
  if (j >= a.ngroups) return;
  uint64_t base = j;
  if (K >= 2) base = ((base >> a.sb0) << (a.sb0 + 1)) | (base & ((1ull << a.sb0) - 1));
  if (K >= 3) base = ((base >> a.sb1) << (a.sb1 + 1)) | (base & ((1ull << a.sb1) - 1));
  double2 x[M];
#pragma unroll
  for (int r = 0; r < M; ++r) {
    const bool own = ((r >> a.gshift) & 1) == a.rank;
    x[r] = own ? loc[base + a.loff[r]] : rem[base + a.loff[r]];
  }
#pragma unroll
  for (int r = 0; r < M; ++r) {
    if (((r >> a.gshift) & 1) != a.rank) continue;
    double2 acc = make_double2(0.0, 0.0);
#pragma unroll
    for (int c = 0; c < M; ++c) acc = cmad(acc, a.u[r * M + c], x[c]);
    loc[base + a.loff[r]] = acc;
  }
}

template <int K>
int launch_shard(const int *targets, const qcw_c64 *U, int rank, double2 *loc, const double2 *rem,
                 int nq, hipStream_t s) {
  ShardArg<K> a;
  constexpr int M = 1 << K;
  for (int e = 0; e < M * M; ++e) a.u[e] = make_double2(U[e].re, U[e].im);
  int gpos = 0;
  for (int j = 0; j < K; ++j)
    if (targets[j] == 1) gpos = j;
  a.gshift = K - 1 - gpos;
  a.rank = rank;
  int lb[2] = {0, 0}, nl = 0;
  for (int j = 0; j < K; ++j)
    if (j != gpos) lb[nl++] = nq - targets[j];  // local bit (same position in the share)
  for (int r = 0; r < M; ++r) {
    uint64_t o = 0;
    for (int j = 0; j < K; ++j)
      if (j != gpos && ((r >> (K - 1 - j)) & 1)) o |= 1ull << (nq - targets[j]);
    a.loff[r] = o;
  }
  a.sb0 = nl > 0 ? std::min(lb[0], nl > 1 ? lb[1] : lb[0]) : 0;
  a.sb1 = nl > 1 ? std::max(lb[0], lb[1]) : 0;
  a.ngroups = 1ull << (nq - 1 - (K - 1));
  const uint64_t blocks = (a.ngroups + kShardBlock - 1) / kShardBlock;
  hipLaunchKernelGGL(shard_kernel<K>, dim3((unsigned)blocks), dim3(kShardBlock), 0, s, loc, rem, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(QCW_EHIP, "shard launch: %s", hipGetErrorString(e));
  return QCW_OK;
}

}  // namespace

}  // namespace qcw

using namespace qcw;

extern "C" int qcw_op_shard(int k, const int *targets, const qcw_c64 *U, int rank_bit,
                            qcw_c64 *psi_local, const qcw_c64 *psi_remote, int nq, void *stream) {
  clear_error();
  if (!U || !targets) return fail(QCW_EINVAL, "NULL argument");
  if (nq < 2 || nq > kMaxQubits) return fail(QCW_EINVAL, "nq=%d outside [2, %d]", nq, kMaxQubits);
  if (rank_bit != 0 && rank_bit != 1) return fail(QCW_EINVAL, "rank_bit=%d is not 0 or 1", rank_bit);
  Geom g;
  int rc = make_geom(nq, k, targets, &g);
  if (rc) return rc;
  const uint64_t bytes = ((uint64_t)1 << (nq - 1)) * sizeof(qcw_c64);
  if ((rc = check_device_range(psi_local, bytes, "psi_local"))) return rc;
  bool global = false;
  for (int j = 0; j < k; ++j) global |= targets[j] == 1;
  hipStream_t s = (hipStream_t)stream;
  if (!global) {
    // the share is an (nq-1)-qubit state whose qubit q is the full state's q+1
    int t[3];
    for (int j = 0; j < k; ++j) t[j] = targets[j] - 1;
    Geom gl;
    if ((rc = make_geom(nq - 1, k, t, &gl))) return rc;
    return launch_sweep(gl, U, psi_local, psi_local, s);
  }
  if ((rc = check_device_range(psi_remote, bytes, "psi_remote"))) return rc;
  const uint64_t a = (uint64_t)(uintptr_t)psi_local, b = (uint64_t)(uintptr_t)psi_remote;
  if (a < b + bytes && b < a + bytes) return fail(QCW_EINVAL, "psi_local and psi_remote overlap");
  double2 *loc = reinterpret_cast<double2 *>(psi_local);
  const double2 *rem = reinterpret_cast<const double2 *>(psi_remote);
  switch (k) {
    case 1: return launch_shard<1>(targets, U, rank_bit, loc, rem, nq, s);
    case 2: return launch_shard<2>(targets, U, rank_bit, loc, rem, nq, s);
    default: return launch_shard<3>(targets, U, rank_bit, loc, rem, nq, s);
  }
}

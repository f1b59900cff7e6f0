// Multiverse density-matrix step (QCWAVE §5): the ensemble average over noisy
// paths (Eqs. rhoE1 and rhoE4), conjugation by the algorithm's gates, and the
// observables the paper tracks.
//
// Layout: rho is 2^nq x 2^nq complex128, row-major, element (n, m) at
// n * 2^nq + m.  Read as a vector it is a 2nq-qubit state whose qubits 1..nq
// are the row qubits and nq+1..2nq the column qubits, so U rho U^dagger is
// the one-gate sweep of U on the row targets followed by the sweep of conj(U)
// on the column targets.
#include <hip/hip_runtime.h>
#include <math.h>
#include <string.h>

#include <algorithm>
#include <utility>
#include <vector>

#include "channel_tiled.h"
#include "qcw_device.h"
#include "qcw_host.h"

namespace qcw {


__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cconj(double2 a) { return make_double2(a.x, -a.y); }

struct DevTerm {
  int32_t nops;
  int32_t bit0, bit1;  // bit positions (nq - qubit) of the operator qubits
  int32_t coef_off;    // first coefficient of this term's table
  double weight;
  double pad;
  double2 k0[4], k1[4];  // 2x2 operators, row-major
};

// Terms sharing a flip mask read the same element of rho: one gather per group.
struct PermGroup {
  uint64_t flip;
  int32_t first, count;
  int32_t n1;   // hits with one operator; they come first in the group
  int32_t pad;
};

// Coefficient tables, built once on the device when a channel is created.
// Single hit: c[(r*2 + c) * 4 + a*2 + e] = K[r][a] conj(K[c][e]), so that
// (K rho K^dagger)_{nm} = sum_{a,e} c[...] rho_{n(a), m(e)}.  Double hit: the
// same with r, c, a, e running over the two qubits' values (16 x 16 entries),
// coefficient K0[r0][a0] K1[r1][a1] conj(K0[c0][e0] K1[c1][e1]).
__global__ void channel_coef_kernel(const DevTerm *__restrict__ terms, int nterms,
                                    double2 *__restrict__ coef) {
  const int t = blockIdx.x;
  if (t >= nterms) return;
  const DevTerm &T = terms[t];
  if (T.nops == 1) {
    for (int i = threadIdx.x; i < 16; i += blockDim.x) {
      const int r = i >> 3 & 1, c = i >> 2 & 1, a = i >> 1 & 1, e = i & 1;
      coef[T.coef_off + i] = cmul(T.k0[r * 2 + a], cconj(T.k0[c * 2 + e]));
    }
  } else {
    for (int i = threadIdx.x; i < 256; i += blockDim.x) {
      const int ri = i >> 6 & 3, ci = i >> 4 & 3, ai = i >> 2 & 3, ei = i & 3;
      const double2 kr = cmul(T.k0[(ri >> 1) * 2 + (ai >> 1)], T.k1[(ri & 1) * 2 + (ai & 1)]);
      const double2 kc = cmul(T.k0[(ci >> 1) * 2 + (ei >> 1)], T.k1[(ci & 1) * 2 + (ei & 1)]);
      coef[T.coef_off + i] = cmul(kr, cconj(kc));
    }
  }
}

// A wave-uniform double, pinned to a scalar register: the entries of a
// coefficient table are read once per wave (scalar loads) and chosen between
// as values.  (Left alone, the compiler turns the choice into a per-lane
// address and a vector load per term, whose wait also drains the gathers.)
__device__ __forceinline__ double uniform_double(double v) {
  const int lo = __builtin_amdgcn_readfirstlane(__double2loint(v));
  const int hi = __builtin_amdgcn_readfirstlane(__double2hiint(v));
  return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double2 pick4(const double2 (&c)[4], int r, int cc) {
  double2 e[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) e[k] = make_double2(uniform_double(c[k].x), uniform_double(c[k].y));
  const double2 lo = cc ? e[1] : e[0];
  const double2 hi = cc ? e[3] : e[2];
  return r ? hi : lo;
}

constexpr int kChanBatch = 8;             // flip-mask groups gathered together
constexpr int kChanTableMaxQubits = 16;   // the interleaved row/column index fits 32 bits

constexpr int kChanTableMaxTerms = 256;   // permutation terms staged in LDS (34 KiB)

// One output element x = n * 2^nq + m of the channel.  With TAB, ctab holds
// every permutation term's coefficients in LDS (term t: c0 at 8t .. 8t+3, c1
// at 8t+4 .. 8t+7), followed by the terms' doubled bit positions (int2 per
// term), and each hit's coefficient is one LDS read at a 2-bit index.  Without it, coefficients are chosen between scalar values: with
// scalar selects when the hit's qubits are the same in every lane, else with
// vector selects (each of which costs a move as well).
template <bool TAB>
__device__ __forceinline__ void channel_one(
    const double2 *__restrict__ rho, double2 *__restrict__ out, int nq, double p_keep,
    const PermGroup *__restrict__ groups, int ngroups, const PermTerm *__restrict__ perm,
    const DevTerm *__restrict__ terms, int nterms, const double2 *__restrict__ coef, uint64_t x,
    uint32_t lane_bits, const double2 *ctab, int nperm) {
  const uint64_t N = 1ull << nq;
  const uint64_t n = x >> nq, m = x & (N - 1);
  const uint32_t n32 = (uint32_t)n, m32 = (uint32_t)m;  // nq <= kRhoMaxQubits < 32
  // Bits of n and m outside lane_bits are the same in every lane of the
  // wavefront: a hit on such qubits has one coefficient per wave, chosen
  // from the first lane's n and m with scalar selects.
  const uint32_t nu = __builtin_amdgcn_readfirstlane(n32);
  const uint32_t mu = __builtin_amdgcn_readfirstlane(m32);
  const double2 r = rho[x];
  double2 acc_all = make_double2(p_keep * r.x, p_keep * r.y);
  // With TAB (nq <= 16): bits 2b+1 and 2b of nm are bit b of n and of m, so
  // (nm >> 2b) & 3 indexes a hit's coefficient table at its qubit bit b.
  const uint32_t nm = TAB ? (spread16(n32) << 1) | spread16(m32) : 0u;
  // Sum of the coefficients of the hits in flip-mask group g at (n, m).
  auto group_sum = [&](int g) {
    const int first = groups[g].first, count = groups[g].count;
    double2 cs = make_double2(0.0, 0.0);
    if (TAB) {
      // One-operator hits, then two-operator hits; each hit's bit positions
      // (doubled, as shifts into nm) come from the LDS table too, so a hit
      // costs no scalar load, and its 2-bit index is one bit-field extract.
      const int2 *dsc = reinterpret_cast<const int2 *>(ctab + 8 * nperm);
      const int mid = first + groups[g].n1;
      for (int t = first; t < mid; ++t) {
        const double2 c = ctab[8 * t + ((nm >> dsc[t].x) & 3u)];
        cs.x += c.x;
        cs.y += c.y;
      }
      for (int t = mid; t < first + count; ++t) {
        const int2 b = dsc[t];
        const double2 c = cmul(ctab[8 * t + ((nm >> b.x) & 3u)], ctab[8 * t + 4 + ((nm >> b.y) & 3u)]);
        cs.x += c.x;
        cs.y += c.y;
      }
      return cs;
    }
    for (int t = first; t < first + count; ++t) {
      const PermTerm &T = perm[t];
      double2 c;
      if ((((1u << T.bit0) | (T.nops == 2 ? 1u << T.bit1 : 0u)) & lane_bits) == 0) {
        // wave-uniform hit
        c = pick4(T.c0, (int)((nu >> T.bit0) & 1u), (int)((mu >> T.bit0) & 1u));
        if (T.nops == 2)
          c = cmul(c, pick4(T.c1, (int)((nu >> T.bit1) & 1u), (int)((mu >> T.bit1) & 1u)));
      } else {
        c = pick4(T.c0, (int)((n32 >> T.bit0) & 1u), (int)((m32 >> T.bit0) & 1u));
        if (T.nops == 2)
          c = cmul(c, pick4(T.c1, (int)((n32 >> T.bit1) & 1u), (int)((m32 >> T.bit1) & 1u)));
      }
      cs.x += c.x;
      cs.y += c.y;
    }
    return cs;
  };
  // Groups are sorted by flip mask, so only the first can be flip-free; it
  // takes rho[x] itself.
  int gstart = 0;
  if (ngroups > 0 && groups[0].flip == 0) {
    acc_all = cmad(acc_all, group_sum(0), r);
    gstart = 1;
  }
  // The gathers of kChanBatch flip-mask groups are issued before their
  // coefficients are summed, so several are in flight per thread; the
  // accumulation still runs in group order.
  for (int g0 = gstart; g0 < ngroups; g0 += kChanBatch) {
    double2 v[kChanBatch];
#pragma unroll
    for (int k = 0; k < kChanBatch; ++k) {
      if (g0 + k < ngroups) {
        const uint32_t flip = (uint32_t)groups[g0 + k].flip;
        v[k] = rho[((uint64_t)(n32 ^ flip) << nq) | (m32 ^ flip)];
      }
    }
#pragma unroll
    for (int k = 0; k < kChanBatch; ++k) {
      if (g0 + k < ngroups) acc_all = cmad(acc_all, group_sum(g0 + k), v[k]);
    }
  }
  for (int t = 0; t < nterms; ++t) {
    const DevTerm &T = terms[t];
    double2 acc = make_double2(0.0, 0.0);
    // A hit on qubits outside lane_bits has one coefficient block per wave:
    // its index comes from the first lane's n and m, so every lane reads the
    // same entries (one cache line per load instead of up to four or
    // sixteen; same values, same operations; the branch is the same in every
    // lane).
    if (T.nops == 1) {
      const int b = T.bit0;
      const uint64_t n0 = n & ~(1ull << b), m0 = m & ~(1ull << b);
      auto hit = [&](const double2 *C) {
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
          for (int e = 0; e < 2; ++e)
            acc = cmad(acc, C[a * 2 + e],
                       rho[((n0 | ((uint64_t)a << b)) << nq) | (m0 | ((uint64_t)e << b))]);
      };
      if (((1u << b) & lane_bits) == 0)
        hit(coef + T.coef_off + (((nu >> b) & 1u) * 2 + ((mu >> b) & 1u)) * 4);
      else
        hit(coef + T.coef_off + (((n32 >> b) & 1u) * 2 + ((m32 >> b) & 1u)) * 4);
    } else {
      const int b0 = T.bit0, b1 = T.bit1;
      const uint64_t clr = ~((1ull << b0) | (1ull << b1));
      const uint64_t n0 = n & clr, m0 = m & clr;
      auto hit = [&](const double2 *C) {
#pragma unroll
        for (int ai = 0; ai < 4; ++ai) {
          const uint64_t nn = n0 | ((uint64_t)(ai >> 1) << b0) | ((uint64_t)(ai & 1) << b1);
#pragma unroll
          for (int ei = 0; ei < 4; ++ei) {
            const uint64_t mm = m0 | ((uint64_t)(ei >> 1) << b0) | ((uint64_t)(ei & 1) << b1);
            acc = cmad(acc, C[ai * 4 + ei], rho[(nn << nq) | mm]);
          }
        }
      };
      auto block = [&](uint32_t nv, uint32_t mv) {
        const uint32_t ri = ((nv >> b0) & 1u) * 2 + ((nv >> b1) & 1u);
        const uint32_t ci = ((mv >> b0) & 1u) * 2 + ((mv >> b1) & 1u);
        return coef + T.coef_off + (ri * 4 + ci) * 16;
      };
      if ((((1u << b0) | (1u << b1)) & lane_bits) == 0)
        hit(block(nu, mu));
      else
        hit(block(n32, m32));
    }
    acc_all.x = __fma_rn(T.weight, acc.x, acc_all.x);
    acc_all.y = __fma_rn(T.weight, acc.y, acc_all.y);
  }
  out[x] = acc_all;
}

constexpr int kChanThreadBits = 8;
constexpr int kChanThreads = 1 << kChanThreadBits;
constexpr int kChanChunkBits = 4;              // 2^4 columns = one 256-byte chunk
constexpr int kXcdBits = 3;                    // 8 XCDs
constexpr unsigned kChanMaxBlocks = 1u << 20;  // a multiple of the XCD count

// Element (n * 2^nq + m) that thread `threadIdx.x` of virtual block vb
// handles: a bijection of the 4^nq elements.  A permutation-type term links
// (n, m) with (n ^ f, m ^ f), and both share o = (n >> L) ^ (m >> L) for
// L = kChanChunkBits.  Ids run over one o at a time (all 2^nq rows, each at
// its 2^L-column chunk), so a block's gathers stay among the 2^(nq+L)
// elements of its o.  Blocks are dealt to the XCDs in turn, so block vb takes
// an o congruent to vb mod 8: each XCD works through its own o values, whose
// elements stay in that XCD's L2.  Below 8 values of o, plain order.
__device__ __forceinline__ uint64_t channel_element(uint64_t vb, int nq) {
  constexpr int L = kChanChunkBits;
  if (nq < L + kXcdBits) return vb * kChanThreads + threadIdx.x;
  const int gb = nq + L - kChanThreadBits;  // log2 of the blocks per value of o
  const uint64_t j = vb >> kXcdBits;
  const uint64_t o = ((j >> gb) << kXcdBits) | (vb & ((1u << kXcdBits) - 1));
  const uint64_t i = (o << (nq + L)) | ((j & ((1ull << gb) - 1)) << kChanThreadBits) | threadIdx.x;
  const uint64_t n = (i >> L) & ((1ull << nq) - 1);
  const uint64_t m = ((o ^ (n >> L)) << L) | (i & ((1ull << L) - 1));
  return (n << nq) | m;
}

// Bits of n and m that can differ between the 64 lanes of a wavefront under
// channel_element's order: in the cache order, lanes vary the low L bits of m
// and the two lowest bits of n (a subset); in plain order a wavefront spans
// 64 consecutive elements, the low six bits of n * 2^nq + m.
__device__ __forceinline__ uint32_t channel_lane_bits(int nq) {
  constexpr int L = kChanChunkBits;
  if (nq >= L + kXcdBits) return (1u << L) - 1;
  const uint32_t vm = (1u << (nq < 6 ? nq : 6)) - 1;
  const uint32_t vn = nq < 6 ? (1u << (6 - nq)) - 1 : 0u;
  return vm | vn;
}

// out = p rho + sum_t w_t K_t rho K_t^dagger, one thread per output element
// (blocks stride over the virtual blocks).  Permutation-type terms first, one
// gather per flip-mask group; then the dense terms from their coefficient
// tables.
template <bool TAB>
__global__ __launch_bounds__(kChanThreads) void channel_kernel(
    const double2 *__restrict__ rho, double2 *__restrict__ out, int nq, double p_keep,
    const PermGroup *__restrict__ groups, int ngroups, const PermTerm *__restrict__ perm, int nperm,
    const DevTerm *__restrict__ terms, int nterms, const double2 *__restrict__ coef) {
  extern __shared__ double2 ctab[];
  if (TAB) {
    for (int e = threadIdx.x; e < 8 * nperm; e += kChanThreads) {
      const PermTerm &T = perm[e >> 3];
      ctab[e] = (e & 4) ? T.c1[e & 3] : T.c0[e & 3];
    }
    int2 *dsc = reinterpret_cast<int2 *>(ctab + 8 * nperm);
    for (int t = threadIdx.x; t < nperm; t += kChanThreads)
      dsc[t] = make_int2(2 * perm[t].bit0, 2 * perm[t].bit1);
    __syncthreads();
  }
  const uint64_t NN = 1ull << (2 * nq);
  const uint64_t nvb = (NN + kChanThreads - 1) / kChanThreads;
  for (uint64_t vb = blockIdx.x; vb < nvb; vb += gridDim.x) {
    if (vb * kChanThreads + threadIdx.x >= NN) continue;
    channel_one<TAB>(rho, out, nq, p_keep, groups, ngroups, perm, terms, nterms, coef,
                     channel_element(vb, nq), channel_lane_bits(nq), ctab, nperm);
  }
}

// ------------------------------------------------------------------ observables
constexpr int kObsThreads = 256;

template <int NV>
__device__ void block_sum(double (&v)[NV], double *red) {
  // fixed-order tree over the block (deterministic)
  for (int i = 0; i < NV; ++i) {
    red[threadIdx.x] = v[i];
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
      if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
      __syncthreads();
    }
    v[i] = red[0];
    __syncthreads();
  }
}

// Partial sums per block: trace (re, im), sum |rho|^2 (= Tr rho^2 for a
// Hermitian rho), and <psi0|rho|psi0> (re).  Each thread takes kObsPerThread
// elements per step (grid-strided), all loaded before any is summed, so
// several loads are in flight per lane; the grid depends only on nq, so the
// summation order, and the result, is the same on every call.
constexpr int kObsPerThread = 8;
constexpr int kObsMaxBlocks = 2048;

static int obs_blocks(int nq) {
  const uint64_t NN = 1ull << (2 * nq);
  const uint64_t b = NN / ((uint64_t)kObsThreads * kObsPerThread);
  return (int)std::max<uint64_t>(1, std::min<uint64_t>(b, kObsMaxBlocks));
}

__global__ __launch_bounds__(kObsThreads) void obs_partial_kernel(const double2 *__restrict__ rho,
                                                                  int nq,
                                                                  const double2 *__restrict__ psi0,
                                                                  double *__restrict__ partial) {
  __shared__ double red[kObsThreads];
  const uint64_t N = 1ull << nq, NN = N * N;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  double v[4] = {0, 0, 0, 0};
  for (uint64_t x0 = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; x0 < NN;
       x0 += stride * kObsPerThread) {
    double2 r[kObsPerThread];
#pragma unroll
    for (int k = 0; k < kObsPerThread; ++k) {
      const uint64_t x = x0 + k * stride;
      r[k] = x < NN ? rho[x] : make_double2(0.0, 0.0);
    }
#pragma unroll
    for (int k = 0; k < kObsPerThread; ++k) {
      const uint64_t x = x0 + k * stride;
      if (x >= NN) break;
      const uint64_t n = x >> nq, m = x & (N - 1);
      if (n == m) {
        v[0] += r[k].x;
        v[1] += r[k].y;
      }
      v[2] += r[k].x * r[k].x + r[k].y * r[k].y;
      if (psi0) {
        const double2 f = cmul(cmul(cconj(psi0[n]), r[k]), psi0[m]);
        v[3] += f.x;
      }
    }
  }
  block_sum<4>(v, red);
  if (threadIdx.x == 0)
    for (int i = 0; i < 4; ++i) partial[blockIdx.x * 4 + i] = v[i];
}

// Records of four partial sums (part[4 r + v]) summed block by block: block b
// takes records [b * per, (b + 1) * per) (thread t the records t, t + 256,
// ... of that range), then the block's fixed tree; the grid depends only on
// the record count, so the result is the same on every call.
__global__ __launch_bounds__(kObsThreads) void obs_records_kernel(const double *__restrict__ part,
                                                                  uint64_t nrec, uint64_t per,
                                                                  double *__restrict__ partial) {
  __shared__ double red[kObsThreads];
  double v[4] = {0, 0, 0, 0};
  const uint64_t b0 = (uint64_t)blockIdx.x * per, b1 = b0 + per < nrec ? b0 + per : nrec;
  for (uint64_t i = b0 + threadIdx.x; i < b1; i += kObsThreads)
    for (int k = 0; k < 4; ++k) v[k] += part[i * 4 + k];
  block_sum<4>(v, red);
  if (threadIdx.x == 0)
    for (int k = 0; k < 4; ++k) partial[blockIdx.x * 4 + k] = v[k];
}

// One block per (qubit, component): P = Tr[sigma^(q) rho], read off the 2x2
// blocks of rho on that qubit.
__global__ __launch_bounds__(kObsThreads) void obs_polar_kernel(const double2 *__restrict__ rho,
                                                                int nq,
                                                                double *__restrict__ out) {
  __shared__ double red[kObsThreads];
  const int q = blockIdx.x / 3 + 1, comp = blockIdx.x % 3;
  const int b = nq - q;
  const uint64_t N = 1ull << nq, st = 1ull << b;
  // Rows n = tid, tid + blockDim.x, ... in ascending order; eight rows'
  // loads are issued before their terms are added (in that order), since
  // every element lies in a row of its own.
  constexpr int U = 8;
  double v[1] = {0};
  for (uint64_t n0 = threadIdx.x; n0 < N; n0 += U * (uint64_t)blockDim.x) {
    double t[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const uint64_t n = n0 + (uint64_t)u * blockDim.x;
      t[u] = 0.0;
      if (n >= N) continue;
      if (comp == 2) {
        const double d = rho[n * N + n].x;
        t[u] = ((n >> b) & 1) ? -d : d;
      } else if (!((n >> b) & 1)) {
        const double2 a = rho[n * N + (n | st)];   // <n|rho|n'>, qubit q: 0 -> 1
        const double2 c = rho[(n | st) * N + n];   // <n'|rho|n>
        t[u] = comp == 0 ? (a.x + c.x) : (c.y - a.y);
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) v[0] += t[u];
  }
  block_sum<1>(v, red);
  if (threadIdx.x == 0) out[4 + blockIdx.x] = v[0];
}

// One block per parameter of the two-qubit form (§5, the footnote to the
// density-matrix paragraph) of qubits at state bits ba (first) and bb: block
// b < 3 gives P1 = Tr[(sigma_(b+1) x 1) rho], b < 6 P2 = Tr[(1 x sigma) rho],
// then C_ij = Tr[(sigma_i x sigma_j) rho] row-major.  Operators are coded
// 0 = 1, 1 = X, 2 = Y, 3 = Z.  Each Pauli row l has one nonzero, in column
// l (1, Z) or 1 - l (X, Y), so Tr[(A x B) rho] = sum over rows (la, lb) and
// over the other bits s of A[la][ka] B[lb][kb] rho[(s, ka, kb), (s, la, lb)].
__device__ __forceinline__ int pauli_col(int op, int l) { return op == 1 || op == 2 ? 1 - l : l; }
__device__ __forceinline__ double2 pauli_coef(int op, int l) {
  switch (op) {
    case 2: return make_double2(0.0, l ? 1.0 : -1.0);  // [[0, -i], [i, 0]]
    case 3: return make_double2(l ? -1.0 : 1.0, 0.0);
    default: return make_double2(1.0, 0.0);
  }
}
__global__ __launch_bounds__(kObsThreads) void pair_pol_kernel(const double2 *__restrict__ rho,
                                                               int nq, int ba, int bb,
                                                               double *__restrict__ out) {
  __shared__ double red[kObsThreads];
  const int b = blockIdx.x;
  const int A = b < 3 ? b + 1 : b < 6 ? 0 : 1 + (b - 6) / 3;
  const int B = b < 3 ? 0 : b < 6 ? b - 2 : 1 + (b - 6) % 3;
  const int lo = ba < bb ? ba : bb, hi = ba < bb ? bb : ba;
  const uint64_t N = 1ull << nq, rest = 1ull << (nq - 2);
  double v[1] = {0};
  for (uint64_t s = threadIdx.x; s < rest; s += blockDim.x) {
    uint64_t base = ((s >> lo) << (lo + 1)) | (s & ((1ull << lo) - 1));
    base = ((base >> hi) << (hi + 1)) | (base & ((1ull << hi) - 1));
#pragma unroll
    for (int l = 0; l < 4; ++l) {
      const int la = l >> 1, lb = l & 1;
      const int ka = pauli_col(A, la), kb = pauli_col(B, lb);
      const double2 ca = pauli_coef(A, la), cb = pauli_coef(B, lb);
      const double2 c = make_double2(ca.x * cb.x - ca.y * cb.y, ca.x * cb.y + ca.y * cb.x);
      const uint64_t row = base | ((uint64_t)ka << ba) | ((uint64_t)kb << bb);
      const uint64_t col = base | ((uint64_t)la << ba) | ((uint64_t)lb << bb);
      const double2 x = rho[row * N + col];
      v[0] += c.x * x.x - c.y * x.y;  // Re(c x); c is 1, -1, i or -i
    }
  }
  block_sum<1>(v, red);
  if (threadIdx.x == 0) out[b] = v[0];
}

// The blocks' partial sums, in a fixed order (thread t takes blocks t,
// t + kObsThreads, ..., then the block's fixed tree), so the result does not
// depend on timing.  One block of kObsThreads threads.
__global__ __launch_bounds__(kObsThreads) void obs_final_kernel(const double *__restrict__ partial,
                                                                int nblocks, double *__restrict__ out,
                                                                int has_psi) {
  __shared__ double red[kObsThreads];
  double s[4] = {0, 0, 0, 0};
  for (int b = threadIdx.x; b < nblocks; b += kObsThreads)
    for (int i = 0; i < 4; ++i) s[i] += partial[b * 4 + i];
  block_sum<4>(s, red);
  if (threadIdx.x == 0) {
    out[0] = s[0];
    out[1] = s[1];
    out[2] = s[2];
    out[3] = has_psi ? sqrt(fmax(s[3], 0.0)) : NAN;
  }
}

}  // namespace qcw

using namespace qcw;

struct qcw_channel {
  int nq = 0;
  double p_keep = 0;
  int nterms = 0;
  int ngroups = 0;
  int nperm = 0;               // permutation terms (in groups)
  DevTerm *terms_d = nullptr;  // dense terms
  double2 *coef_d = nullptr;
  PermGroup *groups_d = nullptr;
  PermTerm *perm_d = nullptr;
  int64_t flops_gather = 0;       // real FP64 operations per output element, gather kernel
  TiledChannel *tiled = nullptr;  // tiled plan (permutation terms only, 7 <= nq <= 15)
  int force_gather = 0;           // run the gather kernel even with a tiled plan
  int tiled_generic = 0;          // run the generic tiled kernel even with a compiled one
  double *obs_part = nullptr;     // partial observables of qcw_channel_step_obs (on first use)
  size_t obs_part_bytes = 0;
};

namespace {
void channel_free(qcw_channel *c) {
  (void)hipFree(c->terms_d);
  (void)hipFree(c->coef_d);
  (void)hipFree(c->groups_d);
  (void)hipFree(c->perm_d);
  (void)hipFree(c->obs_part);
  tiled_channel_free(c->tiled);
  delete c;
}
}  // namespace

extern "C" {

int qcw_rho_conjugate(int k, const int *targets, const qcw_c64 *U, qcw_c64 *rho, int nq,
                      void *stream) {
  clear_error();
  if (nq < 1 || nq > kRhoMaxQubits) return fail(QCW_EINVAL, "nq=%d outside [1, %d]", nq, kRhoMaxQubits);
  if (!U) return fail(QCW_EINVAL, "matrix is NULL");
  Geom g;
  int rc = make_geom(nq, k, targets, &g);
  if (rc) return rc;
  if ((rc = check_device_range(rho, ((uint64_t)1 << (2 * nq)) * sizeof(qcw_c64), "rho"))) return rc;
  int t2[3], t3[3];
  for (int j = 0; j < k; ++j) {
    t2[j] = targets[j];       // row qubits = superket qubits 1..nq
    t3[j] = targets[j] + nq;  // column qubits = superket qubits nq+1..2nq
  }
  Geom gr, gc;
  if ((rc = make_geom(2 * nq, k, t2, &gr)) || (rc = make_geom(2 * nq, k, t3, &gc))) return rc;
  // One pass of LDS tiles from 2 * kConjTileBits superket qubits on (bit for
  // bit the two sweeps below), else a sweep on the rows and one on the columns.
  if (2 * nq >= kConjTileBits) return launch_conjugate(nq, k, targets, U, rho, (hipStream_t)stream);
  const int mm = 1 << (2 * k);
  qcw_c64 Uc[64];
  for (int i = 0; i < mm; ++i) Uc[i] = {U[i].re, -U[i].im};
  if ((rc = launch_sweep(gr, U, rho, rho, (hipStream_t)stream))) return rc;
  return launch_sweep(gc, Uc, rho, rho, (hipStream_t)stream);
}

namespace {

// Validates the terms and splits them into permutation-type terms (with
// their flip masks, sorted by flip mask, one-operator terms first within a
// mask, otherwise in input order) and general terms.
int parse_terms(int nq, const qcw_kraus_term *terms, int nterms, const qcw_c64 *mats, int64_t nmats,
                std::vector<DevTerm> &dt, std::vector<std::pair<uint64_t, PermTerm>> &pt) {
  if (nq < 1 || nq > kRhoMaxQubits) return fail(QCW_EINVAL, "nq=%d outside [1, %d]", nq, kRhoMaxQubits);
  if (nterms < 0 || (nterms > 0 && (!terms || !mats))) return fail(QCW_EINVAL, "bad term list");
  for (int i = 0; i < nterms; ++i) {
    const qcw_kraus_term &t = terms[i];
    if (t.nops < 1 || t.nops > 2) return fail(QCW_EINVAL, "term %d: nops=%d outside {1, 2}", i, t.nops);
    double2 k[2][4];
    for (int j = 0; j < t.nops; ++j) {
      if (t.q[j] < 1 || t.q[j] > nq) return fail(QCW_EINVAL, "term %d: qubit %d outside [1, %d]", i, t.q[j], nq);
      if (t.mat[j] < 0 || t.mat[j] + 4 > nmats) return fail(QCW_EINVAL, "term %d: matrix outside mats", i);
      for (int e = 0; e < 4; ++e) k[j][e] = make_double2(mats[t.mat[j] + e].re, mats[t.mat[j] + e].im);
    }
    if (t.nops == 2 && t.q[0] == t.q[1]) return fail(QCW_EINVAL, "term %d: repeated qubit", i);
    const int bit0 = nq - t.q[0], bit1 = t.nops == 2 ? nq - t.q[1] : 0;
    // Permutation type: per operator, exactly one nonzero per row, in different
    // columns (s = 0: diagonal, s = 1: anti-diagonal).
    auto nz = [](double2 a) { return a.x != 0.0 || a.y != 0.0; };
    int swaps[2] = {0, 0};
    bool perm_type = true;
    for (int j = 0; j < t.nops; ++j) {
      const bool diag = nz(k[j][0]) && nz(k[j][3]) && !nz(k[j][1]) && !nz(k[j][2]);
      const bool anti = nz(k[j][1]) && nz(k[j][2]) && !nz(k[j][0]) && !nz(k[j][3]);
      perm_type = perm_type && (diag || anti);
      swaps[j] = anti;
    }
    if (perm_type) {
      PermTerm p;
      memset(&p, 0, sizeof(p));
      p.nops = t.nops;
      p.bit0 = bit0;
      p.bit1 = bit1;
      for (int j = 0; j < t.nops; ++j) {
        double2 *cj = j == 0 ? p.c0 : p.c1;
        for (int r = 0; r < 2; ++r)
          for (int c = 0; c < 2; ++c) {
            const double2 a = k[j][r * 2 + (r ^ swaps[j])], b = k[j][c * 2 + (c ^ swaps[j])];
            double2 v = make_double2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
            if (j == 0) v = make_double2(t.weight * v.x, t.weight * v.y);
            cj[r * 2 + c] = v;
          }
      }
      const uint64_t flip = ((uint64_t)swaps[0] << bit0) | (t.nops == 2 ? (uint64_t)swaps[1] << bit1 : 0);
      pt.emplace_back(flip, p);
    } else {
      DevTerm d;
      memset(&d, 0, sizeof(d));
      d.nops = t.nops;
      d.weight = t.weight;
      d.bit0 = bit0;
      d.bit1 = bit1;
      for (int e = 0; e < 4; ++e) {
        d.k0[e] = k[0][e];
        if (t.nops == 2) d.k1[e] = k[1][e];
      }
      dt.push_back(d);
    }
  }
  // Group the permutation terms by flip mask, one-operator hits first in
  // each group (stable: otherwise input order).
  std::stable_sort(pt.begin(), pt.end(),
                   [](const std::pair<uint64_t, PermTerm> &a, const std::pair<uint64_t, PermTerm> &b) {
                     if (a.first != b.first) return a.first < b.first;
                     return a.second.nops < b.second.nops;
                   });
  return QCW_OK;
}

// U as a monomial matrix of the gate's local basis (one nonzero entry in
// each column, in distinct rows): U |l> = u_l |table[l]>.
bool gate_monomial(int k, const Geom &g, const qcw_c64 *U, OutPerm *p) {
  const int m = 1 << k;
  memset(p, 0, sizeof(*p));
  p->k = k;
  for (int j = 0; j < k; ++j) p->bits[j] = g.bit[j];
  bool used[8] = {};
  p->unit = 1;
  for (int col = 0; col < m; ++col) {
    int row = -1;
    for (int r = 0; r < m; ++r) {
      const qcw_c64 v = U[r * m + col];
      if (v.re != 0.0 || v.im != 0.0) {
        if (row >= 0) return false;
        row = r;
      }
    }
    if (row < 0 || used[row]) return false;
    used[row] = true;
    p->table[col] = (uint8_t)row;
    p->ur[col] = U[row * m + col].re;
    p->ui[col] = U[row * m + col].im;
    if (p->ur[col] != 1.0 || p->ui[col] != 0.0) p->unit = 0;
  }
  return true;
}

// A gate that is not monomial, with every target among the four lowest
// qubits (state bits 0..3): the compiled kernel applies it to each tile's
// outputs, its matrix passed with the launch.
bool gate_low(int k, const Geom &g, OutPerm *p) {
  memset(p, 0, sizeof(*p));
  p->k = k;
  p->general = 1;
  for (int j = 0; j < k; ++j) {
    if (g.bit[j] > 3) return false;
    p->bits[j] = g.bit[j];
  }
  return true;
}

// The folded form of a gate for the compiled kernel (monomial, or general on
// the lowest qubits), or false.
bool gate_fold(int k, const Geom &g, const qcw_c64 *U, OutPerm *p) {
  return gate_monomial(k, g, U, p) || gate_low(k, g, p);
}

}  // namespace

int qcw_channel_create(qcw_channel **out, int nq, double p_keep, const qcw_kraus_term *terms,
                       int nterms, const qcw_c64 *mats, int64_t nmats) {
  clear_error();
  if (!out) return fail(QCW_EINVAL, "out is NULL");
  *out = nullptr;
  std::vector<DevTerm> dt;
  std::vector<std::pair<uint64_t, PermTerm>> pt;  // (flip mask, term)
  {
    const int rc = parse_terms(nq, terms, nterms, mats, nmats, dt, pt);
    if (rc) return rc;
  }
  std::vector<PermGroup> groups;
  std::vector<PermTerm> perm;
  int64_t flops = 2;  // p_keep * rho
  for (size_t i = 0; i < pt.size(); ++i) {
    if (groups.empty() || groups.back().flip != pt[i].first) {
      groups.push_back(PermGroup{pt[i].first, (int32_t)i, 0, 0, 0});
      flops += 8;  // one complex multiply-add per group
    }
    ++groups.back().count;
    if (pt[i].second.nops == 1) ++groups.back().n1;
    perm.push_back(pt[i].second);
    flops += pt[i].second.nops == 1 ? 2 : 8;  // sum of the coefficient (and its product)
  }
  int64_t ncoef = 0;
  for (DevTerm &d : dt) {
    d.coef_off = (int32_t)ncoef;
    ncoef += d.nops == 1 ? 16 : 256;
    flops += (d.nops == 1 ? 4 : 16) * 8 + 4;
  }
  qcw_channel *c = new qcw_channel();
  c->nq = nq;
  c->p_keep = p_keep;
  c->nterms = (int)dt.size();
  c->ngroups = (int)groups.size();
  c->nperm = (int)perm.size();
  c->flops_gather = flops;
  if (!groups.empty()) {
    if (hipMalloc(&c->groups_d, sizeof(PermGroup) * groups.size()) != hipSuccess ||
        hipMalloc(&c->perm_d, sizeof(PermTerm) * perm.size()) != hipSuccess ||
        hipMemcpy(c->groups_d, groups.data(), sizeof(PermGroup) * groups.size(),
                  hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(c->perm_d, perm.data(), sizeof(PermTerm) * perm.size(), hipMemcpyHostToDevice) !=
            hipSuccess) {
      (void)hipGetLastError();
      channel_free(c);
      return fail(QCW_ENOMEM, "channel terms upload failed");
    }
  }
  if (!dt.empty()) {
    if (hipMalloc(&c->terms_d, sizeof(DevTerm) * dt.size()) != hipSuccess ||
        hipMalloc(&c->coef_d, sizeof(double2) * ncoef) != hipSuccess ||
        hipMemcpy(c->terms_d, dt.data(), sizeof(DevTerm) * dt.size(), hipMemcpyHostToDevice) !=
            hipSuccess) {
      (void)hipGetLastError();
      channel_free(c);
      return fail(QCW_ENOMEM, "channel terms upload failed");
    }
    hipLaunchKernelGGL(channel_coef_kernel, dim3((unsigned)dt.size()), dim3(256), 0, nullptr,
                       c->terms_d, (int)dt.size(), c->coef_d);
    if (hipGetLastError() != hipSuccess || hipDeviceSynchronize() != hipSuccess) {
      channel_free(c);
      return fail(QCW_EHIP, "channel coefficient kernel failed");
    }
  }
  if (dt.empty()) {
    const int rc = tiled_channel_create(nq, p_keep, pt, &c->tiled);
    if (rc) {
      channel_free(c);
      return rc;
    }
  }
  *out = c;
  return QCW_OK;
}

int qcw_channel_apply(const qcw_channel *c, const qcw_c64 *rho_in, qcw_c64 *rho_out, void *stream) {
  clear_error();
  if (!c) return fail(QCW_EINVAL, "channel is NULL");
  const uint64_t NN = 1ull << (2 * c->nq);
  const uint64_t bytes = NN * sizeof(qcw_c64);
  const uint64_t a = (uint64_t)(uintptr_t)rho_in, b = (uint64_t)(uintptr_t)rho_out;
  if (a < b + bytes && b < a + bytes) return fail(QCW_EINVAL, "rho_in and rho_out overlap");
  int rc;
  if ((rc = check_device_range(rho_in, bytes, "rho_in")) || (rc = check_device_range(rho_out, bytes, "rho_out")))
    return rc;
  const unsigned blocks = (unsigned)std::min<uint64_t>((NN + kChanThreads - 1) / kChanThreads, kChanMaxBlocks);
  TimedLaunch t(QCW_KERNEL_CHANNEL, (hipStream_t)stream);
  const double2 *in = reinterpret_cast<const double2 *>(rho_in);
  double2 *o = reinterpret_cast<double2 *>(rho_out);
  if (c->tiled && !c->force_gather)
    return tiled_channel_apply(c->tiled, in, o, (hipStream_t)stream, c->tiled_generic != 0);
  if (c->nperm > 0 && c->nperm <= kChanTableMaxTerms && c->nq <= kChanTableMaxQubits)
    hipLaunchKernelGGL(channel_kernel<true>, dim3(blocks), dim3(kChanThreads),
                       (sizeof(double2) * 8 + sizeof(int) * 2) * c->nperm, (hipStream_t)stream, in,
                       o, c->nq, c->p_keep,
                       c->groups_d, c->ngroups, c->perm_d, c->nperm, c->terms_d, c->nterms, c->coef_d);
  else
    hipLaunchKernelGGL(channel_kernel<false>, dim3(blocks), dim3(kChanThreads), 0,
                       (hipStream_t)stream, in, o, c->nq, c->p_keep, c->groups_d, c->ngroups,
                       c->perm_d, c->nperm, c->terms_d, c->nterms, c->coef_d);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(QCW_EHIP, "channel launch: %s", hipGetErrorString(e));
  return QCW_OK;
}

int qcw_channel_apply_gate(const qcw_channel *c, const qcw_c64 *rho_in, qcw_c64 *rho_out, int k,
                           const int *targets, const qcw_c64 *U, void *stream) {
  clear_error();
  if (!c) return fail(QCW_EINVAL, "channel is NULL");
  if (!U) return fail(QCW_EINVAL, "U is NULL");
  Geom g;
  int rc = make_geom(c->nq, k, targets, &g);
  if (rc) return rc;
  OutPerm p;
  if (c->tiled && !c->force_gather && !c->tiled_generic && gate_fold(k, g, U, &p) &&
      tiled_channel_perm_ready(c->tiled, p)) {
    const uint64_t bytes = (1ull << (2 * c->nq)) * sizeof(qcw_c64);
    const uint64_t a = (uint64_t)(uintptr_t)rho_in, b = (uint64_t)(uintptr_t)rho_out;
    if (a < b + bytes && b < a + bytes) return fail(QCW_EINVAL, "rho_in and rho_out overlap");
    if ((rc = check_device_range(rho_in, bytes, "rho_in")) || (rc = check_device_range(rho_out, bytes, "rho_out")))
      return rc;
    TimedLaunch t(QCW_KERNEL_CHANNEL, (hipStream_t)stream);
    return tiled_channel_apply_perm(c->tiled, p, reinterpret_cast<const double2 *>(rho_in),
                                    reinterpret_cast<double2 *>(rho_out), (hipStream_t)stream,
                                    reinterpret_cast<const double *>(U));
  }
  if ((rc = qcw_channel_apply(c, rho_in, rho_out, stream))) return rc;
  return qcw_rho_conjugate(k, targets, U, rho_out, c->nq, stream);
}

int qcw_channel_step_obs(qcw_channel *c, const qcw_c64 *rho_in, qcw_c64 *rho_out, int k,
                         const int *targets, const qcw_c64 *U, const qcw_c64 *psi0,
                         double *obs, void *stream) {
  clear_error();
  if (!c) return fail(QCW_EINVAL, "channel is NULL");
  if (!obs) return fail(QCW_EINVAL, "obs is NULL");
  const int nq = c->nq;
  const uint64_t N = 1ull << nq, bytes = N * N * sizeof(qcw_c64);
  int rc;
  if ((rc = check_device_range(obs, (4 + 3 * (size_t)nq) * sizeof(double), "obs"))) return rc;
  if (psi0 && (rc = check_device_range(psi0, N * sizeof(qcw_c64), "psi0"))) return rc;
  OutPerm p;
  bool folded = false;
  if (k != 0) {
    if (!U) return fail(QCW_EINVAL, "U is NULL");
    Geom g;
    if ((rc = make_geom(nq, k, targets, &g))) return rc;
    folded = gate_fold(k, g, U, &p);  // a gate the compiled kernel can take
  }
  hipStream_t s = (hipStream_t)stream;
  const bool fused = c->tiled && !c->force_gather && !c->tiled_generic && (k == 0 || folded) &&
                     tiled_channel_obs_ready(c->tiled, folded ? &p : nullptr, psi0 != nullptr);
  const uint64_t records = fused ? tiled_channel_obs_records(c->tiled) : (uint64_t)obs_blocks(nq);
  // the kernel's records are first summed by up to kObsMaxBlocks blocks
  const uint64_t nred = fused ? std::min<uint64_t>(records, kObsMaxBlocks) : 0;
  const size_t need = (records + nred) * 4 * sizeof(double);
  if (c->obs_part_bytes < need) {
    // the previous buffer may still be read by this channel's queued work
    if (c->obs_part && hipDeviceSynchronize() != hipSuccess) return fail(QCW_EHIP, "observables buffer sync");
    (void)hipFree(c->obs_part);
    c->obs_part = nullptr;
    c->obs_part_bytes = 0;
    if (hipMalloc(&c->obs_part, need) != hipSuccess) {
      (void)hipGetLastError();
      return fail(QCW_ENOMEM, "observables buffer of %zu bytes", need);
    }
    c->obs_part_bytes = need;
  }
  const double2 *in = reinterpret_cast<const double2 *>(rho_in);
  double2 *out = reinterpret_cast<double2 *>(rho_out);
  const double2 *ps = reinterpret_cast<const double2 *>(psi0);
  if (fused) {
    const uint64_t a = (uint64_t)(uintptr_t)rho_in, b = (uint64_t)(uintptr_t)rho_out;
    if (a < b + bytes && b < a + bytes) return fail(QCW_EINVAL, "rho_in and rho_out overlap");
    if ((rc = check_device_range(rho_in, bytes, "rho_in")) || (rc = check_device_range(rho_out, bytes, "rho_out")))
      return rc;
    {
      TimedLaunch t(QCW_KERNEL_CHANNEL, s);
      rc = tiled_channel_apply_obs(c->tiled, folded ? &p : nullptr, in, out, ps, c->obs_part, s,
                                   reinterpret_cast<const double *>(U));
    }
    if (rc) return rc;
  } else {
    rc = k == 0 ? qcw_channel_apply(c, rho_in, rho_out, stream)
                : qcw_channel_apply_gate(c, rho_in, rho_out, k, targets, U, stream);
    if (rc) return rc;
    hipLaunchKernelGGL(obs_partial_kernel, dim3((unsigned)records), dim3(kObsThreads), 0, s, out, nq,
                       ps, c->obs_part);
  }
  if (fused) {
    double *red = c->obs_part + records * 4;
    const uint64_t per = (records + nred - 1) / nred;
    hipLaunchKernelGGL(obs_records_kernel, dim3((unsigned)nred), dim3(kObsThreads), 0, s, c->obs_part,
                       records, per, red);
    hipLaunchKernelGGL(obs_final_kernel, dim3(1), dim3(kObsThreads), 0, s, red, (int)nred, obs,
                       psi0 ? 1 : 0);
  } else {
    hipLaunchKernelGGL(obs_final_kernel, dim3(1), dim3(kObsThreads), 0, s, c->obs_part, (int)records, obs,
                       psi0 ? 1 : 0);
  }
  // the polarisations read only the 2 x 2 blocks on each qubit
  hipLaunchKernelGGL(obs_polar_kernel, dim3(3 * nq), dim3(kObsThreads), 0, s, out, nq, obs);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(QCW_EHIP, "step observables: %s", hipGetErrorString(e));
  return QCW_OK;
}

int qcw_channel_destroy(qcw_channel *c) {
  clear_error();
  if (c) channel_free(c);
  return QCW_OK;
}

int64_t qcw_channel_flops_per_element(const qcw_channel *c) {
  if (!c) return -1;
  return c->tiled && !c->force_gather ? tiled_channel_flops(c->tiled) : c->flops_gather;
}

int qcw_debug_channel_plan(qcw_channel *c, int kernel, int32_t *info) {
  clear_error();
  if (!c || !info) return fail(QCW_EINVAL, "channel or info is NULL");
  if (kernel > 2) return fail(QCW_EINVAL, "kernel choice %d outside [-1, 2]", kernel);
  if (kernel >= 0) {
    c->force_gather = kernel == 1 ? 1 : 0;
    c->tiled_generic = kernel == 2 ? 1 : 0;
  }
  TiledSummary sm{};
  tiled_channel_summary(c->tiled, &sm);
  const bool tiled = c->tiled && !c->force_gather;
  const bool spec = tiled && sm.specialized && !c->tiled_generic;
  const int32_t v[17] = {c->tiled ? 1 : 0, tiled ? 0 : 1, sm.e0, sm.e1,
                         sm.partners, sm.staged, sm.direct, sm.own_staged, sm.reads, sm.groups,
                         sm.segments, sm.etouch_segments, sm.real, spec ? 1 : 0,
                         tiled ? (spec ? sm.spec_grid : sm.grid) : 0,
                         tiled ? (spec ? sm.spec_regs : sm.regs) : 0,
                         sm.specialized ? tiled_channel_compiler_version() : 0};
  memcpy(info, v, sizeof(v));
  return QCW_OK;
}

int qcw_debug_channel_source(int nq, const qcw_kraus_term *terms, int nterms, const qcw_c64 *mats,
                             int64_t nmats, int gate_k, const int *gate_targets,
                             const qcw_c64 *gate_U, int observables, int compile, char *buf,
                             size_t cap, size_t *len, size_t *code_bytes,
                             int32_t *compiler_version) {
  clear_error();
  if (compiler_version) *compiler_version = tiled_channel_compiler_version();
  if (!len) return fail(QCW_EINVAL, "len is NULL");
  if (compile && !code_bytes) return fail(QCW_EINVAL, "code_bytes is NULL");
  std::vector<DevTerm> dt;
  std::vector<std::pair<uint64_t, PermTerm>> pt;
  int rc = parse_terms(nq, terms, nterms, mats, nmats, dt, pt);
  if (rc) return rc;
  OutPerm perm;
  bool with_gate = false;
  if (gate_k != 0) {
    Geom g;
    if ((rc = make_geom(nq, gate_k, gate_targets, &g))) return rc;
    if (!gate_U) return fail(QCW_EINVAL, "gate_U is NULL");
    with_gate = gate_fold(gate_k, g, gate_U, &perm);
  }
  *len = 0;
  if (gate_k != 0 && !with_gate) {  // neither monomial nor on the lowest qubits: no kernel of its own
    if (buf && cap > 0) buf[0] = 0;
    if (compile) *code_bytes = 0;
    return QCW_OK;
  }
  const std::string src = dt.empty() ? tiled_channel_source(nq, pt, with_gate ? &perm : nullptr,
                                                           observables != 0)
                                     : std::string();
  *len = src.size();
  if (buf && cap > 0) {
    const size_t n = std::min(cap - 1, src.size());
    memcpy(buf, src.data(), n);
    buf[n] = 0;
  }
  if (compile) {
    *code_bytes = 0;
    if (!src.empty() && (rc = tiled_channel_compile_check(src, code_bytes))) return rc;
  }
  return QCW_OK;
}

int qcw_rho_pair_polarization(const qcw_c64 *rho, int nq, int qa, int qb, double *out,
                              void *stream) {
  clear_error();
  if (nq < 2 || nq > kRhoMaxQubits) return fail(QCW_EINVAL, "nq=%d outside [2, %d]", nq, kRhoMaxQubits);
  if (qa < 1 || qa > nq || qb < 1 || qb > nq || qa == qb)
    return fail(QCW_EINVAL, "qubits (%d, %d): need two distinct qubits in [1, %d]", qa, qb, nq);
  int rc = check_device_range(rho, ((uint64_t)1 << (2 * nq)) * sizeof(qcw_c64), "rho");
  if (rc || (rc = check_device_range(out, 15 * sizeof(double), "out"))) return rc;
  hipLaunchKernelGGL(pair_pol_kernel, dim3(15), dim3(kObsThreads), 0, (hipStream_t)stream,
                     reinterpret_cast<const double2 *>(rho), nq, nq - qa, nq - qb, out);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(QCW_EHIP, "pair polarisation: %s", hipGetErrorString(e));
  return QCW_OK;
}

}  // extern "C"

namespace {

// Device scratch of qcw_rho_observables (partial sums, outputs, psi0): one
// per device, sized for the largest state, allocated on first use and kept
// (freeing it would synchronise the device on every call).  The lock is
// held from the first launch to the copy's completion, so concurrent calls
// do not share it.
std::mutex g_obs_mu;
std::map<int, double *> g_obs_scratch;
constexpr size_t kObsScratchBytes = sizeof(double) * (kObsMaxBlocks * 4 + 4 + 3 * kRhoMaxQubits) +
                                    sizeof(qcw_c64) * ((size_t)1 << kRhoMaxQubits);

int obs_scratch(double **out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) {
    (void)hipGetLastError();
    return fail(QCW_EHIP, "cannot query the device");
  }
  auto it = g_obs_scratch.find(dev);
  if (it != g_obs_scratch.end()) {
    *out = it->second;
    return QCW_OK;
  }
  double *d = nullptr;
  if (hipMalloc(&d, kObsScratchBytes) != hipSuccess) {
    (void)hipGetLastError();
    return fail(QCW_ENOMEM, "observables scratch");
  }
  g_obs_scratch[dev] = d;
  *out = d;
  return QCW_OK;
}

}  // namespace

extern "C" {

int qcw_rho_observables(const qcw_c64 *rho, int nq, const qcw_c64 *psi0_host, double *out_host,
                        void *stream) {
  clear_error();
  if (nq < 1 || nq > kRhoMaxQubits) return fail(QCW_EINVAL, "nq=%d outside [1, %d]", nq, kRhoMaxQubits);
  if (!out_host) return fail(QCW_EINVAL, "out_host is NULL");
  int rc = check_device_range(rho, ((uint64_t)1 << (2 * nq)) * sizeof(qcw_c64), "rho");
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  const int nout = 4 + 3 * nq;
  const size_t N = (size_t)1 << nq;
  std::lock_guard<std::mutex> lk(g_obs_mu);
  double *scratch = nullptr;  // partials, outputs, then psi0
  if ((rc = obs_scratch(&scratch))) return rc;
  const int nblocks = obs_blocks(nq);
  double *partial = scratch, *out = scratch + nblocks * 4;
  double2 *psi_d = psi0_host ? reinterpret_cast<double2 *>(out + nout) : nullptr;
  hipError_t e = hipSuccess;
  if (psi0_host) e = hipMemcpyAsync(psi_d, psi0_host, N * sizeof(qcw_c64), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(obs_partial_kernel, dim3(nblocks), dim3(kObsThreads), 0, s,
                       reinterpret_cast<const double2 *>(rho), nq, psi_d, partial);
    hipLaunchKernelGGL(obs_polar_kernel, dim3(3 * nq), dim3(kObsThreads), 0, s,
                       reinterpret_cast<const double2 *>(rho), nq, out);
    hipLaunchKernelGGL(obs_final_kernel, dim3(1), dim3(kObsThreads), 0, s, partial, nblocks, out,
                       psi0_host ? 1 : 0);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipMemcpyAsync(out_host, out, sizeof(double) * nout, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return fail(QCW_EHIP, "observables: %s", hipGetErrorString(e));
  return QCW_OK;
}

}  // extern "C"

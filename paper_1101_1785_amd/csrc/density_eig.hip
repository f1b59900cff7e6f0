// Eigenvalue-based observables of the multiverse density matrix (QCWAVE §5,
// the classical-limit discussion): eigenvalues, von Neumann entropy, the
// fidelity Tr sqrt(sqrt(rho0) rho sqrt(rho0)) against a mixed reference, and
// the partial trace for subsystem quantities.
//
// Hermitian eigensolver: parallel cyclic Jacobi, one workgroup per matrix,
// the matrix (and eigenvectors) in LDS, n = 2^nq <= 64.  Each step applies
// n/2 disjoint rotations (round-robin pairing): for a pair (p, q) with
// c = A_pq = |c| e^{i phi}, the unitary J = diag(1, e^{-i phi}) R(theta) on
// rows/columns p, q, with the classical real rotation angle chosen from the
// diagonal entries and |c|, zeroes A_pq.  Because the pairs are disjoint, J is
// block diagonal, and A <- J^H A J splits into independent 2 x 2 blocks
// (rows p, q of one pair, columns p', q' of another): one LDS pass per step.
//
// Batched launches are persistent: block b takes matrices b, b + grid, ...;
// the kernels need no memory beyond their inputs and outputs.
#include <hip/hip_runtime.h>
#include <float.h>
#include <math.h>

#include <map>
#include <mutex>
#include <tuple>

#include "qcw_host.h"

namespace qcw {

constexpr int kEigMaxN = 64;
constexpr int kEigMaxThreads = 256;
constexpr int kEigChunk = 8;  // rows or columns per step when forming K (fidelity)

// Threads per block for an n x n matrix: a step updates (n/2)^2 blocks of
// 2 x 2 entries, 1024 at n = 64 (four per thread), 256 at n = 32.
static int eig_threads(int n) { return n >= 32 ? 256 : 64; }

__device__ __forceinline__ double2 zmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 zconj(double2 a) { return make_double2(a.x, -a.y); }
__device__ __forceinline__ double2 zadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 zscale(double s, double2 a) { return make_double2(s * a.x, s * a.y); }
// c1 a + s1 b
__device__ __forceinline__ double2 zlin(double c1, double2 a, double s1, double2 b) {
  return make_double2(c1 * a.x + s1 * b.x, c1 * a.y + s1 * b.y);
}

struct Rot {
  double c, s, t, ac;  // cos, sin, tan of the angle; |A_pq|
  double2 e;           // e^{i phi}
  int p, q;
};

// Round-robin pairing for step `st` of a sweep over n (even) indices: index
// 0 stays, the others rotate; pair k = (pos[k], pos[n-1-k]).
__device__ __forceinline__ void rr_pair(int n, int st, int k, int *p, int *q) {
  auto at = [&](int i) { return i == 0 ? 0 : 1 + (i - 1 + st) % (n - 1); };
  int a = at(k), b = at(n - 1 - k);
  *p = a < b ? a : b;
  *q = a < b ? b : a;
}

// Sum of one value per thread over the block, in a fixed tree order (the
// same result on every run); every thread receives it.
__device__ double block_sum(double v, double *red) {
  const int tid = threadIdx.x;
  red[tid] = v;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (tid < s) red[tid] += red[tid + s];
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}

// Element (i, j) of the Hermitian part (M + M^dagger) / 2 of a row-major n x n
// matrix in global memory.
__device__ __forceinline__ double2 herm_at(const double2 *__restrict__ M, int n, int i, int j) {
  const double2 a = M[i * n + j], b = M[j * n + i];
  return make_double2(0.5 * (a.x + b.x), 0.5 * (a.y - b.y));
}

// Diagonalises the n x n Hermitian matrix A (row stride lda) in LDS;
// accumulates the eigenvectors as the columns of V (row stride ldv) when
// V != nullptr.  Sweeps until the off-diagonal Frobenius norm squared is at
// most 1e-30 of the matrix norm squared, or 40 sweeps.  n even, 2 <= n <= 64.
__device__ void jacobi_lds(double2 *A, int lda, double2 *V, int ldv, int n, Rot *rot, double *red) {
  const int tid = threadIdx.x, nt = blockDim.x, h = n / 2;
  if (V)
    for (int i = tid; i < n * n; i += nt)
      V[(i / n) * ldv + i % n] = make_double2((i / n) == (i % n) ? 1.0 : 0.0, 0.0);
  double loc = 0;
  for (int i = tid; i < n * n; i += nt) {
    const double2 a = A[(i / n) * lda + i % n];
    loc += a.x * a.x + a.y * a.y;
  }
  const double norm2 = block_sum(loc, red);
  for (int sweep = 0; sweep < 40; ++sweep) {
    loc = 0;
    for (int i = tid; i < n * n; i += nt)
      if ((i / n) != (i % n)) {
        const double2 a = A[(i / n) * lda + i % n];
        loc += a.x * a.x + a.y * a.y;
      }
    const double off2 = block_sum(loc, red);
    if (off2 <= 1e-30 * norm2 || off2 == 0.0) break;
    for (int st = 0; st < n - 1; ++st) {
      // rotation parameters from the current matrix
      for (int k = tid; k < h; k += nt) {
        int p, q;
        rr_pair(n, st, k, &p, &q);
        const double2 c = A[p * lda + q];
        const double ac = sqrt(c.x * c.x + c.y * c.y);
        Rot r;
        r.p = p;
        r.q = q;
        r.ac = ac;
        if (ac < 1e-300) {
          r.t = 0.0;
          r.c = 1.0;
          r.s = 0.0;
          r.e = make_double2(1.0, 0.0);
        } else {
          const double app = A[p * lda + p].x, aqq = A[q * lda + q].x;
          const double theta = (aqq - app) / (2.0 * ac);
          // the smaller root of t^2 + 2 theta t - 1 = 0 (1 / (2 theta) once
          // theta^2 would overflow)
          r.t = fabs(theta) > 1e150 ? 0.5 / theta
                                    : (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
          r.c = 1.0 / sqrt(r.t * r.t + 1.0);
          r.s = r.t * r.c;
          r.e = make_double2(c.x / ac, c.y / ac);
        }
        rot[k] = r;
      }
      __syncthreads();
      // A <- J^H A J, one 2 x 2 block (rows p, q of pair k; columns p2, q2 of
      // pair k2) per work item, k <= k2.  Rows: row_p' = c row_p - s e row_q,
      // row_q' = s row_p + c e row_q; columns: col_p' = c col_p - s conj(e) col_q,
      // col_q' = s col_p + c conj(e) col_q.  The block (k2, k) is the conjugate
      // transpose, written as such, so A stays exactly Hermitian; a diagonal
      // block (k = k2) becomes diag(A_pp - t |A_pq|, A_qq + t |A_pq|), which
      // is what the rotation makes of it in exact arithmetic.
      for (int w = tid; w < h * h; w += nt) {
        const int k = w / h, k2 = w % h;
        if (k > k2) continue;
        const Rot r = rot[k];
        double2 *rp = A + r.p * lda, *rq = A + r.q * lda;
        if (k == k2) {
          rp[r.p] = make_double2(rp[r.p].x - r.t * r.ac, 0.0);
          rq[r.q] = make_double2(rq[r.q].x + r.t * r.ac, 0.0);
          rp[r.q] = make_double2(0.0, 0.0);
          rq[r.p] = make_double2(0.0, 0.0);
          continue;
        }
        const Rot r2 = rot[k2];
        const double2 a = rp[r2.p], b = rp[r2.q], c = rq[r2.p], d = rq[r2.q];
        const double2 ec = zmul(r.e, c), ed = zmul(r.e, d);
        const double2 a1 = zlin(r.c, a, -r.s, ec), c1 = zlin(r.s, a, r.c, ec);
        const double2 b1 = zlin(r.c, b, -r.s, ed), d1 = zlin(r.s, b, r.c, ed);
        const double2 e2 = zconj(r2.e);
        const double2 eb = zmul(e2, b1), ed1 = zmul(e2, d1);
        const double2 pp = zlin(r2.c, a1, -r2.s, eb), pq = zlin(r2.s, a1, r2.c, eb);
        const double2 qp = zlin(r2.c, c1, -r2.s, ed1), qq = zlin(r2.s, c1, r2.c, ed1);
        rp[r2.p] = pp;
        rp[r2.q] = pq;
        rq[r2.p] = qp;
        rq[r2.q] = qq;
        A[r2.p * lda + r.p] = zconj(pp);
        A[r2.q * lda + r.p] = zconj(pq);
        A[r2.p * lda + r.q] = zconj(qp);
        A[r2.q * lda + r.q] = zconj(qq);
      }
      if (V) {
        for (int w = tid; w < n * h; w += nt) {
          const Rot r = rot[w % h];
          double2 *vi = V + (w / h) * ldv;
          const double2 vp = vi[r.p], vq = vi[r.q];
          const double2 eq = zmul(zconj(r.e), vq);
          vi[r.p] = zlin(r.c, vp, -r.s, eq);
          vi[r.q] = zlin(r.s, vp, r.c, eq);
        }
      }
      __syncthreads();
    }
  }
}

// Batched eigenvalues and entropies: matrix m at rho + m * stride (n x n,
// its Hermitian part is diagonalised); eig[m * n ...] ascending and
// entropy[m] = -sum lambda log2 lambda over lambda > 0 (entropy may be NULL).
__global__ __launch_bounds__(kEigMaxThreads) void eig_batch_kernel(
    const double2 *__restrict__ rho, int64_t stride, int n, int64_t count,
    double *__restrict__ eig, double *__restrict__ entropy) {
  extern __shared__ double2 A[];  // n * n
  __shared__ Rot rot[kEigMaxN / 2];
  __shared__ double red[kEigMaxThreads];
  __shared__ double ev[kEigMaxN];
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int64_t m = blockIdx.x; m < count; m += gridDim.x) {
    const double2 *R = rho + m * stride;
    for (int i = tid; i < n * n; i += nt) A[i] = herm_at(R, n, i / n, i % n);
    __syncthreads();
    jacobi_lds(A, n, nullptr, 0, n, rot, red);
    for (int i = tid; i < n; i += nt) ev[i] = A[i * n + i].x;
    __syncthreads();
    // ascending order by rank (ties broken by index), and the entropy terms
    double loc = 0;
    for (int i = tid; i < n; i += nt) {
      const double v = ev[i];
      int rank = 0;
      for (int j = 0; j < n; ++j) {
        const double u = ev[j];
        rank += (u < v) || (u == v && j < i);
      }
      eig[m * n + rank] = v;
      if (v > 0) loc -= v * log2(v);
    }
    const double S = block_sum(loc, red);  // ends with a barrier: A and ev may be reused
    if (entropy && tid == 0) entropy[m] = S;
  }
}

// Batched fidelity F = Tr sqrt(sqrt(rho0) rho sqrt(rho0)) (§5), pair m =
// (rho + m * rs, rho0 + m * r0s); r0s = 0 shares one reference.
//
// Restricted to the range of rho0: with rho0 = V_r diag(l) V_r^dagger over its
// r eigenvalues above n * eps * l_max, sqrt(rho0) = V_r diag(sqrt l) V_r^dagger,
// so sqrt(rho0) rho sqrt(rho0) = V_r K V_r^dagger with the r x r matrix
// K = W^dagger rho W, W = V_r diag(sqrt l).  Both have the same nonzero
// eigenvalues, and F = sum sqrt(kappa) over K's eigenvalues.  A pure reference
// gives r = 1 and F = sqrt(<psi0|rho|psi0>), the closed form, to rounding.
// Eigenvalues of K at or below r * eps * kappa_max are rounding-level (the
// solver's absolute error is about eps * |K|): they are dropped instead of
// contributing ~sqrt(eps) each.
__global__ __launch_bounds__(kEigMaxThreads) void fidelity_batch_kernel(
    const double2 *__restrict__ rho, int64_t rs, const double2 *__restrict__ rho0, int64_t r0s,
    int n, int64_t count, double *__restrict__ F) {
  extern __shared__ double2 sm[];
  double2 *A = sm;              // n x n, row stride n
  double2 *V = sm + n * n;      // n x n, row stride n
  double2 *C = sm + 2 * n * n;  // kEigChunk * n staging
  __shared__ Rot rot[kEigMaxN / 2];
  __shared__ double red[kEigMaxThreads];
  __shared__ double lam[kEigMaxN], ks[kEigMaxN];
  __shared__ int kidx[kEigMaxN];
  __shared__ int nkeep;
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int64_t m = blockIdx.x; m < count; m += gridDim.x) {
    const double2 *R = rho + m * rs, *R0 = rho0 + m * r0s;
    for (int i = tid; i < n * n; i += nt) A[i] = herm_at(R0, n, i / n, i % n);
    __syncthreads();
    jacobi_lds(A, n, V, n, n, rot, red);
    for (int i = tid; i < n; i += nt) lam[i] = A[i * n + i].x;
    __syncthreads();
    if (tid == 0) {
      double lmax = 0;
      for (int i = 0; i < n; ++i) lmax = fmax(lmax, lam[i]);
      const double tau = n * DBL_EPSILON * lmax;
      int r = 0;
      for (int i = 0; i < n; ++i)
        if (lam[i] > tau && lam[i] > 0) {
          kidx[r] = i;
          ks[r] = sqrt(lam[i]);
          ++r;
        }
      nkeep = r;
    }
    __syncthreads();
    const int r = nkeep;
    if (r == 0) {  // rho0 = 0
      if (tid == 0) F[m] = 0.0;
      __syncthreads();
      continue;
    }
    // W = V[:, kidx] diag(sqrt l) into V's first r columns.  Each thread owns
    // whole rows and moves columns in increasing order; kidx[a] >= a, so no
    // source column is overwritten before it is read.
    for (int i = tid; i < n; i += nt)
      for (int a = 0; a < r; ++a) V[i * n + a] = zscale(ks[a], V[i * n + kidx[a]]);
    __syncthreads();
    // T = H(rho) W into A (n x r), kEigChunk rows of H(rho) at a time through C
    for (int j0 = 0; j0 < n; j0 += kEigChunk) {
      const int rb = min(kEigChunk, n - j0);  // rows of this chunk (n < 8: all of them)
      for (int w = tid; w < rb * n; w += nt) C[w] = herm_at(R, n, j0 + w / n, w % n);
      __syncthreads();
      for (int w = tid; w < rb * r; w += nt) {
        const int jj = w / r, b = w % r;
        double2 acc = make_double2(0.0, 0.0);
        for (int i = 0; i < n; ++i) acc = zadd(acc, zmul(C[jj * n + i], V[i * n + b]));
        A[(j0 + jj) * n + b] = acc;
      }
      __syncthreads();
    }
    // K = W^dagger T, kEigChunk columns at a time through C; each column block
    // of K replaces the (no longer needed) same columns of T.
    for (int b0 = 0; b0 < r; b0 += kEigChunk) {
      const int cb = min(kEigChunk, r - b0);
      for (int w = tid; w < r * cb; w += nt) {
        const int a = w / cb, c = w % cb;
        double2 acc = make_double2(0.0, 0.0);
        for (int j = 0; j < n; ++j) acc = zadd(acc, zmul(zconj(V[j * n + a]), A[j * n + b0 + c]));
        C[a * kEigChunk + c] = acc;
      }
      __syncthreads();
      for (int w = tid; w < r * cb; w += nt) {
        const int a = w / cb, c = w % cb;
        A[a * n + b0 + c] = C[a * kEigChunk + c];
      }
      __syncthreads();
    }
    // Hermitian part of K, padded to an even order rp with a zero row and column
    const int rp = r + (r & 1);
    for (int w = tid; w < rp * rp; w += nt) {
      const int a = w / rp, b = w % rp;
      if (a >= r || b >= r) {
        A[a * n + b] = make_double2(0.0, 0.0);
      } else if (a < b) {
        const double2 x = A[a * n + b], y = A[b * n + a];
        const double2 hv = make_double2(0.5 * (x.x + y.x), 0.5 * (x.y - y.y));
        A[a * n + b] = hv;
        A[b * n + a] = zconj(hv);
      } else if (a == b) {
        A[a * n + a].y = 0.0;
      }
    }
    __syncthreads();
    if (r == 1) {
      if (tid == 0) F[m] = sqrt(fmax(A[0].x, 0.0));
      __syncthreads();
      continue;
    }
    jacobi_lds(A, n, nullptr, 0, rp, rot, red);
    if (tid == 0) {
      double kmax = 0;
      for (int i = 0; i < rp; ++i) kmax = fmax(kmax, A[i * n + i].x);
      const double tau = rp * DBL_EPSILON * kmax;
      double f = 0;
      for (int i = 0; i < rp; ++i) {
        const double kv = A[i * n + i].x;
        if (kv > tau) f += sqrt(kv);
      }
      F[m] = f;
    }
    __syncthreads();
  }
}

// Partial trace: keeps the qubits set in `keep` (bit q-1 for qubit q) and sums
// over the others.  out is 2^nk x 2^nk, nk = popcount(keep); the kept qubits
// keep their relative order (the lowest-numbered kept qubit is the most
// significant bit of the reduced label).
__global__ void ptrace_kernel(const double2 *__restrict__ rho, int nq, uint32_t keep_bits,
                              int nk, double2 *__restrict__ out) {
  const uint64_t nr = 1ull << nk;
  const uint64_t x = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= nr * nr) return;
  const uint64_t a = x / nr, a2 = x % nr;
  const int nt = nq - nk;
  // deposit reduced labels and traced labels into full labels
  auto full = [&](uint64_t kept, uint64_t traced) {
    uint64_t n = 0;
    int ik = nk - 1, it = nt - 1;
    for (int q = 1; q <= nq; ++q) {
      const int bitpos = nq - q;
      uint64_t v;
      if ((keep_bits >> (q - 1)) & 1) {
        v = (kept >> ik) & 1;
        --ik;
      } else {
        v = (traced >> it) & 1;
        --it;
      }
      n |= v << bitpos;
    }
    return n;
  };
  const uint64_t N = 1ull << nq;
  double2 acc = make_double2(0, 0);
  for (uint64_t b = 0; b < (1ull << nt); ++b)
    acc = zadd(acc, rho[full(a, b) * N + full(a2, b)]);
  out[x] = acc;
}

// ------------------------------------------------------------------ host side
namespace {

enum EigKernel { kEigValues = 0, kEigFidelity = 1 };

size_t eig_lds_bytes(EigKernel k, int n) {
  const size_t nn = (size_t)n * n;
  return sizeof(double2) * (k == kEigValues ? nn : 2 * nn + (size_t)kEigChunk * n);
}

const void *eig_fn(EigKernel k) {
  return k == kEigValues ? (const void *)eig_batch_kernel : (const void *)fidelity_batch_kernel;
}

// Persistent grid per (device, kernel, n): resident blocks per CU times CUs.
// Set once under a lock (calls may come from several threads).
int eig_grid(EigKernel k, int n, unsigned *grid) {
  static std::mutex mu;
  static std::map<std::tuple<int, int, int>, unsigned> cache;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) {
    (void)hipGetLastError();
    return fail(QCW_EHIP, "cannot query the device");
  }
  std::lock_guard<std::mutex> lk(mu);
  auto key = std::make_tuple(dev, (int)k, n);
  auto it = cache.find(key);
  if (it != cache.end()) {
    *grid = it->second;
    return QCW_OK;
  }
  const size_t lds = eig_lds_bytes(k, n);
  const int nt = eig_threads(n);
  hipError_t e = hipFuncSetAttribute(eig_fn(k), hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)lds);
  int bpc = 0, ncu = 0;
  if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&bpc, eig_fn(k), nt, lds);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(QCW_EHIP, "eigensolver launch shape: %s", hipGetErrorString(e));
  }
  if (bpc < 1) return fail(QCW_EHIP, "eigensolver with %zu B of LDS does not fit a CU", lds);
  *grid = (unsigned)(bpc * ncu);
  cache[key] = *grid;
  return QCW_OK;
}

int launch_eig(const double2 *rho, int64_t stride, int n, int64_t count, double *eig,
               double *entropy, hipStream_t s) {
  if (count == 0) return QCW_OK;
  unsigned grid = 0;
  int rc = eig_grid(kEigValues, n, &grid);
  if (rc) return rc;
  const unsigned blocks = (unsigned)std::min<int64_t>(count, grid);
  hipLaunchKernelGGL(eig_batch_kernel, dim3(blocks), dim3(eig_threads(n)),
                     eig_lds_bytes(kEigValues, n), s, rho, stride, n, count, eig, entropy);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(QCW_EHIP, "eigenvalue launch: %s", hipGetErrorString(e));
  return QCW_OK;
}

int launch_fidelity(const double2 *rho, int64_t rs, const double2 *rho0, int64_t r0s, int n,
                    int64_t count, double *F, hipStream_t s) {
  if (count == 0) return QCW_OK;
  unsigned grid = 0;
  int rc = eig_grid(kEigFidelity, n, &grid);
  if (rc) return rc;
  const unsigned blocks = (unsigned)std::min<int64_t>(count, grid);
  hipLaunchKernelGGL(fidelity_batch_kernel, dim3(blocks), dim3(eig_threads(n)),
                     eig_lds_bytes(kEigFidelity, n), s, rho, rs, rho0, r0s, n, count, F);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(QCW_EHIP, "fidelity launch: %s", hipGetErrorString(e));
  return QCW_OK;
}

// Device landing buffer of the synchronous single-matrix calls: one per
// device, allocated on first use and kept; the lock is held from the launch
// to the copy's completion, so concurrent calls do not share it.
std::mutex g_land_mu;
std::map<int, double *> g_land;
constexpr size_t kLandDoubles = kEigMaxN + 1;

int landing(double **out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) {
    (void)hipGetLastError();
    return fail(QCW_EHIP, "cannot query the device");
  }
  auto it = g_land.find(dev);
  if (it != g_land.end()) {
    *out = it->second;
    return QCW_OK;
  }
  double *d = nullptr;
  if (hipMalloc(&d, sizeof(double) * kLandDoubles) != hipSuccess) {
    (void)hipGetLastError();
    return fail(QCW_ENOMEM, "eigenvalue output buffer");
  }
  g_land[dev] = d;
  *out = d;
  return QCW_OK;
}

int check_batch_args(int nq, int64_t count, int64_t stride, bool stride0_ok, const void *p,
                     const char *what) {
  const int64_t nn = (int64_t)1 << (2 * nq);
  if (stride < nn && !(stride0_ok && stride == 0))
    return fail(QCW_EINVAL, "%s stride %lld below 4^nq = %lld", what, (long long)stride,
                (long long)nn);
  const uint64_t elems = (uint64_t)(count - 1) * (uint64_t)stride + (uint64_t)nn;
  return check_device_range(p, elems * sizeof(qcw_c64), what);
}

}  // namespace

}  // namespace qcw

using namespace qcw;

extern "C" {

int qcw_rho_eigvals_batch(const qcw_c64 *rho, int nq, int64_t count, int64_t stride, double *eig,
                          double *entropy, void *stream) {
  clear_error();
  if (nq < 1 || nq > 6) return fail(QCW_EINVAL, "nq=%d outside [1, 6]", nq);
  if (count < 0) return fail(QCW_EINVAL, "count < 0");
  if (count == 0) return QCW_OK;
  const int n = 1 << nq;
  int rc;
  if ((rc = check_batch_args(nq, count, stride, false, rho, "rho")) ||
      (rc = check_device_range(eig, (uint64_t)count * n * sizeof(double), "eig")) ||
      (entropy && (rc = check_device_range(entropy, (uint64_t)count * sizeof(double), "entropy"))))
    return rc;
  return launch_eig(reinterpret_cast<const double2 *>(rho), stride, n, count, eig, entropy,
                    (hipStream_t)stream);
}

int qcw_rho_fidelity_batch(const qcw_c64 *rho, int64_t rho_stride, const qcw_c64 *rho0,
                           int64_t rho0_stride, int nq, int64_t count, double *fidelity,
                           void *stream) {
  clear_error();
  if (nq < 1 || nq > 6) return fail(QCW_EINVAL, "nq=%d outside [1, 6]", nq);
  if (count < 0) return fail(QCW_EINVAL, "count < 0");
  if (count == 0) return QCW_OK;
  int rc;
  if ((rc = check_batch_args(nq, count, rho_stride, false, rho, "rho")) ||
      (rc = check_batch_args(nq, count, rho0_stride, true, rho0, "rho0")) ||
      (rc = check_device_range(fidelity, (uint64_t)count * sizeof(double), "fidelity")))
    return rc;
  return launch_fidelity(reinterpret_cast<const double2 *>(rho), rho_stride,
                         reinterpret_cast<const double2 *>(rho0), rho0_stride, 1 << nq, count,
                         fidelity, (hipStream_t)stream);
}

int qcw_rho_eigvals(const qcw_c64 *rho, int nq, double *out_host, void *stream) {
  clear_error();
  if (nq < 1 || nq > 6) return fail(QCW_EINVAL, "nq=%d outside [1, 6]", nq);
  if (!out_host) return fail(QCW_EINVAL, "out_host is NULL");
  const int n = 1 << nq;
  int rc = check_device_range(rho, (uint64_t)n * n * sizeof(qcw_c64), "rho");
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  std::lock_guard<std::mutex> lk(g_land_mu);
  double *d = nullptr;
  if ((rc = landing(&d))) return rc;
  if ((rc = launch_eig(reinterpret_cast<const double2 *>(rho), (int64_t)n * n, n, 1, d, d + n, s)))
    return rc;
  hipError_t e = hipMemcpyAsync(out_host, d, sizeof(double) * (n + 1), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return fail(QCW_EHIP, "eigenvalues: %s", hipGetErrorString(e));
  return QCW_OK;
}

int qcw_rho_fidelity(const qcw_c64 *rho, const qcw_c64 *rho0, int nq, double *out_host,
                     void *stream) {
  clear_error();
  if (nq < 1 || nq > 6) return fail(QCW_EINVAL, "nq=%d outside [1, 6]", nq);
  if (!out_host) return fail(QCW_EINVAL, "out_host is NULL");
  const int n = 1 << nq;
  const uint64_t bytes = (uint64_t)n * n * sizeof(qcw_c64);
  int rc;
  if ((rc = check_device_range(rho, bytes, "rho")) || (rc = check_device_range(rho0, bytes, "rho0")))
    return rc;
  hipStream_t s = (hipStream_t)stream;
  std::lock_guard<std::mutex> lk(g_land_mu);
  double *d = nullptr;
  if ((rc = landing(&d))) return rc;
  if ((rc = launch_fidelity(reinterpret_cast<const double2 *>(rho), 0,
                            reinterpret_cast<const double2 *>(rho0), 0, n, 1, d, s)))
    return rc;
  hipError_t e = hipMemcpyAsync(out_host, d, sizeof(double), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return fail(QCW_EHIP, "fidelity: %s", hipGetErrorString(e));
  return QCW_OK;
}

int qcw_rho_partial_trace(const qcw_c64 *rho, int nq, const int *keep, int nkeep, qcw_c64 *out,
                          void *stream) {
  clear_error();
  if (nq < 1 || nq > kMaxQubits / 2) return fail(QCW_EINVAL, "nq=%d outside [1, 17]", nq);
  if (nkeep < 1 || nkeep > nq || !keep) return fail(QCW_EINVAL, "keep 1..nq qubits");
  uint32_t bits = 0;
  for (int i = 0; i < nkeep; ++i) {
    if (keep[i] < 1 || keep[i] > nq) return fail(QCW_EINVAL, "qubit %d outside [1, %d]", keep[i], nq);
    if ((bits >> (keep[i] - 1)) & 1) return fail(QCW_EINVAL, "qubit %d repeated", keep[i]);
    bits |= 1u << (keep[i] - 1);
  }
  int rc;
  if ((rc = check_device_range(rho, ((uint64_t)1 << (2 * nq)) * sizeof(qcw_c64), "rho")) ||
      (rc = check_device_range(out, ((uint64_t)1 << (2 * nkeep)) * sizeof(qcw_c64), "out")))
    return rc;
  const uint64_t nr2 = 1ull << (2 * nkeep);
  hipLaunchKernelGGL(ptrace_kernel, dim3((unsigned)((nr2 + 255) / 256)), dim3(256), 0,
                     (hipStream_t)stream, reinterpret_cast<const double2 *>(rho), nq, bits, nkeep,
                     reinterpret_cast<double2 *>(out));
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(QCW_EHIP, "partial trace: %s", hipGetErrorString(e));
  return QCW_OK;
}

}  // extern "C"

// Eigenvalue-based observables of the multiverse density matrix (QCWAVE §5,
// the classical-limit discussion): eigenvalues, von Neumann entropy, the
// fidelity Tr sqrt(sqrt(rho0) rho sqrt(rho0)) against a mixed reference, and
// the partial trace for subsystem quantities.
//
// Hermitian eigensolver: parallel cyclic Jacobi in one workgroup, matrix (and
// eigenvectors) in LDS, for n = 2^nq <= 64.  Each step applies n/2 disjoint
// rotations (round-robin pairing): for a pair (p, q) with c = A_pq = |c| e^{i phi},
// the unitary J = diag(1, e^{-i phi}) R(theta) on rows/columns p, q, with the
// classical real rotation angle chosen from the diagonal entries and |c|, zeroes
// A_pq; A <- J^H A J and V <- V J.
#include <hip/hip_runtime.h>
#include <math.h>

#include "qcw_host.h"

namespace qcw {

constexpr int kEigMaxN = 64;
constexpr int kEigThreads = 256;

__device__ __forceinline__ double2 zmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 zconj(double2 a) { return make_double2(a.x, -a.y); }
__device__ __forceinline__ double2 zadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 zscale(double s, double2 a) { return make_double2(s * a.x, s * a.y); }

struct Rot {
  double c, s;
  double2 e;  // e^{i phi}
};

// Round-robin pairing for step `st` of a sweep over n (even) indices: index
// 0 stays, the others rotate; pair k = (pos[k], pos[n-1-k]).
__device__ __forceinline__ void rr_pair(int n, int st, int k, int *p, int *q) {
  auto at = [&](int i) { return i == 0 ? 0 : 1 + (i - 1 + st) % (n - 1); };
  int a = at(k), b = at(n - 1 - k);
  *p = a < b ? a : b;
  *q = a < b ? b : a;
}

// Diagonalises the n x n Hermitian matrix in LDS (A, row-major); accumulates
// eigenvectors in V when V != nullptr.  Runs until the off-diagonal Frobenius
// norm is below tol times the matrix norm, or 40 sweeps.
__device__ void jacobi_lds(double2 *A, double2 *V, int n, Rot *rot, double *red) {
  const int tid = threadIdx.x;
  if (V)
    for (int i = tid; i < n * n; i += blockDim.x)
      V[i] = make_double2((i / n) == (i % n) ? 1.0 : 0.0, 0.0);
  __syncthreads();
  // matrix norm for the stopping test
  double loc = 0;
  for (int i = tid; i < n * n; i += blockDim.x) loc += A[i].x * A[i].x + A[i].y * A[i].y;
  red[tid] = loc;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (tid < s) red[tid] += red[tid + s];
    __syncthreads();
  }
  const double norm2 = red[0];
  __syncthreads();
  for (int sweep = 0; sweep < 40; ++sweep) {
    // off-diagonal norm
    loc = 0;
    for (int i = tid; i < n * n; i += blockDim.x)
      if ((i / n) != (i % n)) loc += A[i].x * A[i].x + A[i].y * A[i].y;
    red[tid] = loc;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
      if (tid < s) red[tid] += red[tid + s];
      __syncthreads();
    }
    const double off2 = red[0];
    __syncthreads();
    if (off2 <= 1e-30 * norm2 || off2 == 0.0) break;
    for (int st = 0; st < n - 1; ++st) {
      // rotation parameters from the current matrix
      for (int k = tid; k < n / 2; k += blockDim.x) {
        int p, q;
        rr_pair(n, st, k, &p, &q);
        const double2 c = A[p * n + q];
        const double ac = sqrt(c.x * c.x + c.y * c.y);
        Rot r;
        if (ac < 1e-300) {
          r.c = 1.0;
          r.s = 0.0;
          r.e = make_double2(1.0, 0.0);
        } else {
          const double app = A[p * n + p].x, aqq = A[q * n + q].x;
          const double theta = (aqq - app) / (2.0 * ac);
          const double t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
          r.c = 1.0 / sqrt(t * t + 1.0);
          r.s = t * r.c;
          r.e = make_double2(c.x / ac, c.y / ac);
        }
        rot[k] = r;
      }
      __syncthreads();
      // rows: row_p' = c row_p - s e row_q ; row_q' = s row_p + c e row_q
      for (int w = tid; w < (n / 2) * n; w += blockDim.x) {
        const int k = w / n, j = w % n;
        int p, q;
        rr_pair(n, st, k, &p, &q);
        const Rot r = rot[k];
        const double2 ap = A[p * n + j], aq = A[q * n + j];
        const double2 eq = zmul(r.e, aq);
        A[p * n + j] = make_double2(r.c * ap.x - r.s * eq.x, r.c * ap.y - r.s * eq.y);
        A[q * n + j] = make_double2(r.s * ap.x + r.c * eq.x, r.s * ap.y + r.c * eq.y);
      }
      __syncthreads();
      // columns: col_p' = c col_p - s conj(e) col_q ; col_q' = s col_p + c conj(e) col_q
      for (int w = tid; w < (n / 2) * n; w += blockDim.x) {
        const int k = w / n, i = w % n;
        int p, q;
        rr_pair(n, st, k, &p, &q);
        const Rot r = rot[k];
        const double2 ec = zconj(r.e);
        {
          const double2 ap = A[i * n + p], aq = A[i * n + q];
          const double2 eq = zmul(ec, aq);
          A[i * n + p] = make_double2(r.c * ap.x - r.s * eq.x, r.c * ap.y - r.s * eq.y);
          A[i * n + q] = make_double2(r.s * ap.x + r.c * eq.x, r.s * ap.y + r.c * eq.y);
        }
        if (V) {
          const double2 vp = V[i * n + p], vq = V[i * n + q];
          const double2 eq = zmul(ec, vq);
          V[i * n + p] = make_double2(r.c * vp.x - r.s * eq.x, r.c * vp.y - r.s * eq.y);
          V[i * n + q] = make_double2(r.s * vp.x + r.c * eq.x, r.s * vp.y + r.c * eq.y);
        }
      }
      __syncthreads();
    }
  }
}

// Eigenvalues (ascending) and entropy in bits: out[0..n-1] = lambda,
// out[n] = -sum lambda log2 lambda over lambda > 0.
__global__ __launch_bounds__(kEigThreads) void eig_kernel(const double2 *__restrict__ rho, int n,
                                                          double *__restrict__ out) {
  extern __shared__ double2 A[];  // n * n
  __shared__ Rot rot[kEigMaxN / 2];
  __shared__ double red[kEigThreads];
  for (int i = threadIdx.x; i < n * n; i += blockDim.x) {
    // Hermitian part, (rho + rho^dagger) / 2
    const int r = i / n, c = i % n;
    const double2 a = rho[i], b = rho[c * n + r];
    A[i] = make_double2(0.5 * (a.x + b.x), 0.5 * (a.y - b.y));
  }
  __syncthreads();
  jacobi_lds(A, nullptr, n, rot, red);
  if (threadIdx.x == 0) {
    double ev[kEigMaxN];
    for (int i = 0; i < n; ++i) ev[i] = A[i * n + i].x;
    for (int i = 1; i < n; ++i) {  // insertion sort, ascending
      const double v = ev[i];
      int j = i - 1;
      while (j >= 0 && ev[j] > v) {
        ev[j + 1] = ev[j];
        --j;
      }
      ev[j + 1] = v;
    }
    double S = 0;
    for (int i = 0; i < n; ++i) {
      out[i] = ev[i];
      if (ev[i] > 0) S -= ev[i] * log2(ev[i]);
    }
    out[n] = S;
  }
}

// Fidelity F = Tr sqrt(sqrt(rho0) rho sqrt(rho0)): eigendecompose rho0 =
// V diag(l) V^dagger, form sqrt(rho0) = V diag(sqrt(max(l, 0))) V^dagger,
// M = sqrt(rho0) rho sqrt(rho0), and sum sqrt(max(mu, 0)) over M's eigenvalues.
__global__ __launch_bounds__(kEigThreads) void fidelity_kernel(const double2 *__restrict__ rho,
                                                               const double2 *__restrict__ rho0,
                                                               int n, double2 *__restrict__ work,
                                                               double *__restrict__ out) {
  extern __shared__ double2 L[];
  double2 *A = L;                 // n*n
  double2 *V = L + n * n;         // n*n
  __shared__ Rot rot[kEigMaxN / 2];
  __shared__ double red[kEigThreads];
  double2 *Sq = work;             // n*n in global memory
  double2 *Tm = work + n * n;     // n*n
  for (int i = threadIdx.x; i < n * n; i += blockDim.x) {
    const int r = i / n, c = i % n;
    const double2 a = rho0[i], b = rho0[c * n + r];
    A[i] = make_double2(0.5 * (a.x + b.x), 0.5 * (a.y - b.y));
  }
  __syncthreads();
  jacobi_lds(A, V, n, rot, red);
  // Sq = V diag(sqrt(l)) V^dagger
  for (int i = threadIdx.x; i < n * n; i += blockDim.x) {
    const int r = i / n, c = i % n;
    double2 acc = make_double2(0, 0);
    for (int k = 0; k < n; ++k) {
      const double l = A[k * n + k].x;
      const double sl = l > 0 ? sqrt(l) : 0.0;
      acc = zadd(acc, zscale(sl, zmul(V[r * n + k], zconj(V[c * n + k]))));
    }
    Sq[i] = acc;
  }
  __syncthreads();
  // Tm = Sq rho
  for (int i = threadIdx.x; i < n * n; i += blockDim.x) {
    const int r = i / n, c = i % n;
    double2 acc = make_double2(0, 0);
    for (int k = 0; k < n; ++k) acc = zadd(acc, zmul(Sq[r * n + k], rho[k * n + c]));
    Tm[i] = acc;
  }
  __syncthreads();
  // A = Tm Sq (Hermitian part)
  for (int i = threadIdx.x; i < n * n; i += blockDim.x) {
    const int r = i / n, c = i % n;
    double2 acc = make_double2(0, 0);
    for (int k = 0; k < n; ++k) acc = zadd(acc, zmul(Tm[r * n + k], Sq[k * n + c]));
    A[i] = acc;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < n * n; i += blockDim.x) {
    const int r = i / n, c = i % n;
    if (r < c) {
      const double2 a = A[i], b = A[c * n + r];
      const double2 h = make_double2(0.5 * (a.x + b.x), 0.5 * (a.y - b.y));
      A[i] = h;
      A[c * n + r] = zconj(h);
    } else if (r == c) {
      A[i].y = 0.0;
    }
  }
  __syncthreads();
  jacobi_lds(A, nullptr, n, rot, red);
  if (threadIdx.x == 0) {
    double F = 0;
    for (int i = 0; i < n; ++i) {
      const double mu = A[i * n + i].x;
      if (mu > 0) F += sqrt(mu);
    }
    out[0] = F;
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

}  // namespace qcw

using namespace qcw;

extern "C" {

int qcw_rho_eigvals(const qcw_c64 *rho, int nq, double *out_host, void *stream) {
  clear_error();
  if (nq < 1 || nq > 6) return fail(QCW_EINVAL, "nq=%d outside [1, 6]", nq);
  if (!out_host) return fail(QCW_EINVAL, "out_host is NULL");
  const int n = 1 << nq;
  int rc = check_device_range(rho, (uint64_t)n * n * sizeof(qcw_c64), "rho");
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  double *d = nullptr;
  if (hipMalloc(&d, sizeof(double) * (n + 1)) != hipSuccess) {
    (void)hipGetLastError();
    return fail(QCW_ENOMEM, "eigenvalue output");
  }
  const size_t lds = (size_t)n * n * sizeof(double2);
  hipError_t e = hipSuccess;
  if (lds > 60 * 1024)
    e = hipFuncSetAttribute((const void *)eig_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)lds);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(eig_kernel, dim3(1), dim3(kEigThreads), lds, s,
                       reinterpret_cast<const double2 *>(rho), n, d);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipMemcpyAsync(out_host, d, sizeof(double) * (n + 1), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  (void)hipFree(d);
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
  char *d = nullptr;
  if (hipMalloc(&d, 2 * bytes + sizeof(double)) != hipSuccess) {
    (void)hipGetLastError();
    return fail(QCW_ENOMEM, "fidelity scratch");
  }
  const size_t lds = 2 * bytes;  // A and V
  hipError_t e = hipSuccess;
  if (lds > 60 * 1024)
    e = hipFuncSetAttribute((const void *)fidelity_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)lds);
  double *dout = reinterpret_cast<double *>(d + 2 * bytes);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(fidelity_kernel, dim3(1), dim3(kEigThreads), lds, s,
                       reinterpret_cast<const double2 *>(rho), reinterpret_cast<const double2 *>(rho0),
                       n, reinterpret_cast<double2 *>(d), dout);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipMemcpyAsync(out_host, dout, sizeof(double), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  (void)hipFree(d);
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

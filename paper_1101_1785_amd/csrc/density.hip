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

#include <vector>

#include "qcw_device.h"
#include "qcw_host.h"

namespace qcw {

constexpr int kRhoMaxQubits = 17;  // 2 * 17 = 34 superket qubits

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cconj(double2 a) { return make_double2(a.x, -a.y); }

struct DevTerm {
  int32_t nops;
  int32_t bit0, bit1;  // bit positions (nq - qubit) of the operator qubits
  int32_t pad;
  double weight;
  double pad2;
  double2 k0[4], k1[4];  // 2x2 operators, row-major
};

// out = p rho + sum_t w_t K_t rho K_t^dagger, one thread per output element.
__global__ __launch_bounds__(256) void channel_kernel(const double2 *__restrict__ rho,
                                                      double2 *__restrict__ out, int nq,
                                                      double p_keep,
                                                      const DevTerm *__restrict__ terms,
                                                      int nterms) {
  const uint64_t NN = 1ull << (2 * nq);
  const uint64_t x = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= NN) return;
  const uint64_t N = 1ull << nq;
  const uint64_t n = x >> nq, m = x & (N - 1);
  const double2 r = rho[x];
  double2 acc_all = make_double2(p_keep * r.x, p_keep * r.y);
  for (int t = 0; t < nterms; ++t) {
    const DevTerm &T = terms[t];
    double2 acc = make_double2(0.0, 0.0);
    if (T.nops == 1) {
      const int b = T.bit0;
      const int rb = (int)((n >> b) & 1), cb = (int)((m >> b) & 1);
      const uint64_t n0 = n & ~(1ull << b), m0 = m & ~(1ull << b);
      for (int a = 0; a < 2; ++a)
        for (int c = 0; c < 2; ++c) {
          const double2 coef = cmul(T.k0[rb * 2 + a], cconj(T.k0[cb * 2 + c]));
          const double2 v = rho[((n0 | ((uint64_t)a << b)) << nq) | (m0 | ((uint64_t)c << b))];
          const double2 p = cmul(coef, v);
          acc.x += p.x;
          acc.y += p.y;
        }
    } else {
      const int b0 = T.bit0, b1 = T.bit1;
      const int r0 = (int)((n >> b0) & 1), r1 = (int)((n >> b1) & 1);
      const int c0 = (int)((m >> b0) & 1), c1 = (int)((m >> b1) & 1);
      const uint64_t clr = ~((1ull << b0) | (1ull << b1));
      const uint64_t n0 = n & clr, m0 = m & clr;
      for (int a0 = 0; a0 < 2; ++a0)
        for (int a1 = 0; a1 < 2; ++a1) {
          const double2 kr = cmul(T.k0[r0 * 2 + a0], T.k1[r1 * 2 + a1]);
          const uint64_t nn = n0 | ((uint64_t)a0 << b0) | ((uint64_t)a1 << b1);
          for (int e0 = 0; e0 < 2; ++e0)
            for (int e1 = 0; e1 < 2; ++e1) {
              const double2 kc = cconj(cmul(T.k0[c0 * 2 + e0], T.k1[c1 * 2 + e1]));
              const uint64_t mm = m0 | ((uint64_t)e0 << b0) | ((uint64_t)e1 << b1);
              const double2 p = cmul(cmul(kr, kc), rho[(nn << nq) | mm]);
              acc.x += p.x;
              acc.y += p.y;
            }
        }
    }
    acc_all.x += T.weight * acc.x;
    acc_all.y += T.weight * acc.y;
  }
  out[x] = acc_all;
}

// ------------------------------------------------------------------ observables
constexpr int kObsBlocks = 256;
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
// Hermitian rho), and <psi0|rho|psi0> (re).
__global__ __launch_bounds__(kObsThreads) void obs_partial_kernel(const double2 *__restrict__ rho,
                                                                  int nq,
                                                                  const double2 *__restrict__ psi0,
                                                                  double *__restrict__ partial) {
  __shared__ double red[kObsThreads];
  const uint64_t N = 1ull << nq, NN = N * N;
  double v[4] = {0, 0, 0, 0};
  for (uint64_t x = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; x < NN;
       x += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t n = x >> nq, m = x & (N - 1);
    const double2 r = rho[x];
    if (n == m) {
      v[0] += r.x;
      v[1] += r.y;
    }
    v[2] += r.x * r.x + r.y * r.y;
    if (psi0) {
      const double2 f = cmul(cmul(cconj(psi0[n]), r), psi0[m]);
      v[3] += f.x;
    }
  }
  block_sum<4>(v, red);
  if (threadIdx.x == 0)
    for (int i = 0; i < 4; ++i) partial[blockIdx.x * 4 + i] = v[i];
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
  double v[1] = {0};
  for (uint64_t n = threadIdx.x; n < N; n += blockDim.x) {
    if (comp == 2) {
      const double d = rho[n * N + n].x;
      v[0] += ((n >> b) & 1) ? -d : d;
    } else if (!((n >> b) & 1)) {
      const double2 a = rho[n * N + (n | st)];   // <n|rho|n'>, qubit q: 0 -> 1
      const double2 c = rho[(n | st) * N + n];   // <n'|rho|n>
      v[0] += comp == 0 ? (a.x + c.x) : (c.y - a.y);
    }
  }
  block_sum<1>(v, red);
  if (threadIdx.x == 0) out[4 + blockIdx.x] = v[0];
}

__global__ void obs_final_kernel(const double *__restrict__ partial, int nblocks,
                                 double *__restrict__ out, int has_psi) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double s[4] = {0, 0, 0, 0};
  for (int b = 0; b < nblocks; ++b)
    for (int i = 0; i < 4; ++i) s[i] += partial[b * 4 + i];
  out[0] = s[0];
  out[1] = s[1];
  out[2] = s[2];
  out[3] = has_psi ? sqrt(fmax(s[3], 0.0)) : NAN;
}

}  // namespace qcw

using namespace qcw;

struct qcw_channel {
  int nq = 0;
  double p_keep = 0;
  int nterms = 0;
  DevTerm *terms_d = nullptr;
};

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
  const int mm = 1 << (2 * k);
  qcw_c64 Uc[64];
  for (int i = 0; i < mm; ++i) Uc[i] = {U[i].re, -U[i].im};
  if ((rc = launch_sweep(gr, U, rho, rho, (hipStream_t)stream))) return rc;
  return launch_sweep(gc, Uc, rho, rho, (hipStream_t)stream);
}

int qcw_channel_create(qcw_channel **out, int nq, double p_keep, const qcw_kraus_term *terms,
                       int nterms, const qcw_c64 *mats, int64_t nmats) {
  clear_error();
  if (!out) return fail(QCW_EINVAL, "out is NULL");
  *out = nullptr;
  if (nq < 1 || nq > kRhoMaxQubits) return fail(QCW_EINVAL, "nq=%d outside [1, %d]", nq, kRhoMaxQubits);
  if (nterms < 0 || (nterms > 0 && (!terms || !mats))) return fail(QCW_EINVAL, "bad term list");
  std::vector<DevTerm> dt(nterms);
  for (int i = 0; i < nterms; ++i) {
    const qcw_kraus_term &t = terms[i];
    if (t.nops < 1 || t.nops > 2) return fail(QCW_EINVAL, "term %d: nops=%d outside {1, 2}", i, t.nops);
    memset(&dt[i], 0, sizeof(DevTerm));
    dt[i].nops = t.nops;
    dt[i].weight = t.weight;
    for (int j = 0; j < t.nops; ++j) {
      if (t.q[j] < 1 || t.q[j] > nq) return fail(QCW_EINVAL, "term %d: qubit %d outside [1, %d]", i, t.q[j], nq);
      if (t.mat[j] < 0 || t.mat[j] + 4 > nmats) return fail(QCW_EINVAL, "term %d: matrix outside mats", i);
      double2 *k = j == 0 ? dt[i].k0 : dt[i].k1;
      for (int e = 0; e < 4; ++e) k[e] = make_double2(mats[t.mat[j] + e].re, mats[t.mat[j] + e].im);
    }
    if (t.nops == 2 && t.q[0] == t.q[1]) return fail(QCW_EINVAL, "term %d: repeated qubit", i);
    dt[i].bit0 = nq - t.q[0];
    dt[i].bit1 = t.nops == 2 ? nq - t.q[1] : 0;
  }
  qcw_channel *c = new qcw_channel();
  c->nq = nq;
  c->p_keep = p_keep;
  c->nterms = nterms;
  if (nterms) {
    if (hipMalloc(&c->terms_d, sizeof(DevTerm) * nterms) != hipSuccess ||
        hipMemcpy(c->terms_d, dt.data(), sizeof(DevTerm) * nterms, hipMemcpyHostToDevice) !=
            hipSuccess) {
      (void)hipGetLastError();
      (void)hipFree(c->terms_d);
      delete c;
      return fail(QCW_ENOMEM, "channel terms upload failed");
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
  const unsigned blocks = (unsigned)((NN + 255) / 256);
  TimedLaunch t(QCW_KERNEL_CHANNEL, (hipStream_t)stream);
  hipLaunchKernelGGL(channel_kernel, dim3(blocks), dim3(256), 0, (hipStream_t)stream,
                     reinterpret_cast<const double2 *>(rho_in), reinterpret_cast<double2 *>(rho_out),
                     c->nq, c->p_keep, c->terms_d, c->nterms);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(QCW_EHIP, "channel launch: %s", hipGetErrorString(e));
  return QCW_OK;
}

int qcw_channel_destroy(qcw_channel *c) {
  clear_error();
  if (c) {
    (void)hipFree(c->terms_d);
    delete c;
  }
  return QCW_OK;
}

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
  double *scratch = nullptr;  // partials, outputs, then psi0
  const size_t bytes = sizeof(double) * (kObsBlocks * 4 + nout) + (psi0_host ? N * sizeof(qcw_c64) : 0);
  if (hipMalloc(&scratch, bytes) != hipSuccess) {
    (void)hipGetLastError();
    return fail(QCW_ENOMEM, "observables scratch");
  }
  double *partial = scratch, *out = scratch + kObsBlocks * 4;
  double2 *psi_d = psi0_host ? reinterpret_cast<double2 *>(out + nout) : nullptr;
  hipError_t e = hipSuccess;
  if (psi0_host) e = hipMemcpyAsync(psi_d, psi0_host, N * sizeof(qcw_c64), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(obs_partial_kernel, dim3(kObsBlocks), dim3(kObsThreads), 0, s,
                       reinterpret_cast<const double2 *>(rho), nq, psi_d, partial);
    hipLaunchKernelGGL(obs_polar_kernel, dim3(3 * nq), dim3(kObsThreads), 0, s,
                       reinterpret_cast<const double2 *>(rho), nq, out);
    hipLaunchKernelGGL(obs_final_kernel, dim3(1), dim3(64), 0, s, partial, kObsBlocks, out,
                       psi0_host ? 1 : 0);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipMemcpyAsync(out_host, out, sizeof(double) * nout, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  (void)hipFree(scratch);
  if (e != hipSuccess) return fail(QCW_EHIP, "observables: %s", hipGetErrorString(e));
  return QCW_OK;
}

}  // extern "C"

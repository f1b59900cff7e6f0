/*
 * Plain FP64 CPU oracle for the QCWAVE gate sweep -- TEST INFRASTRUCTURE ONLY.
 *
 * Only tests, the smoke check and the CPU-baseline leg of the benchmark may
 * load this library.  It shares no code, header or table with the HIP
 * library: it is written from the definitions in QCWAVE (Tabakin &
 * Julia-Diaz, arXiv:1101.1785) and kept deliberately slow and literal.
 *
 * Conventions (paper §2c, Eq. staten): amplitude n of an nq-qubit state sits
 * at offset n, with n = sum_i q_i 2^(nq-i); qubit 1 is the most significant
 * bit, so qubit `is` owns bit nq - is.  Complex numbers are interleaved
 * (re, im) doubles.  A k-qubit gate is an m x m row-major complex matrix
 * (m = 2^k), U[r][c] = <r|U|c>, whose local index r lists the k target
 * qubits' values with the first listed target most significant (§3b, the
 * V_{ij;kl} = <ij|V|kl> definition under Eq. resmat2; the three-target case,
 * whose derivation §3c omits, extends it the same way).
 *
 * Build: gcc -O2 -ffp-contract=off -fopenmp -shared -fPIC (no FMA contraction,
 * scalar code), so every product and sum is rounded as written.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_OK 0
#define ORC_EINVAL -1

static int check_targets(int nq, int k, const int *targets) {
  if (nq < 1 || nq > 40 || k < 1 || k > 3 || k > nq || !targets) return 0;
  for (int j = 0; j < k; ++j) {
    if (targets[j] < 1 || targets[j] > nq) return 0;
    for (int i = 0; i < j; ++i)
      if (targets[i] == targets[j]) return 0;
  }
  return 1;
}

int orc_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

void orc_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

/*
 * One output amplitude of a k-qubit operator, from the algebraic result of
 * §3a Eq. oneopres (k = 1) and §3b Eq. twoopA (k = 2):
 *
 *   C~_n = sum over the target values q' of <q_targets(n)| U |q'> C_{n'},
 *
 * where n' equals n except that the target qubits carry the values q'.
 * `bit[j]` is the bit position of the j-th listed target.
 */
static void out_amp(int k, const int *bit, const double *U, const double *in,
                    uint64_t n, double *re_out, double *im_out) {
  int m = 1 << k;
  /* the row: the target qubits' values in n, first target most significant */
  int r = 0;
  for (int j = 0; j < k; ++j) r = (r << 1) | (int)((n >> bit[j]) & 1u);
  /* n with every target qubit set to 0 */
  uint64_t rest = n;
  for (int j = 0; j < k; ++j) rest &= ~((uint64_t)1 << bit[j]);
  double re = 0.0, im = 0.0;
  for (int c = 0; c < m; ++c) {
    uint64_t src = rest;
    for (int j = 0; j < k; ++j)
      if ((c >> (k - 1 - j)) & 1) src |= (uint64_t)1 << bit[j];
    double ur = U[2 * (r * m + c)], ui = U[2 * (r * m + c) + 1];
    double xr = in[2 * src], xi = in[2 * src + 1];
    double pr = ur * xr - ui * xi;
    double pi = ur * xi + ui * xr;
    re = re + pr;
    im = im + pi;
  }
  *re_out = re;
  *im_out = im;
}

/* psi_out = Op_k(U; targets) psi_in, out of place (the paper's
 * psi_f = Op1[U, is, psi_0], §3a footnote; Op2 §3b; Op3 §3c). */
int orc_apply(int nq, int k, const int *targets, const double *U,
              const double *in, double *out) {
  if (!check_targets(nq, k, targets) || !U || !in || !out || in == out)
    return ORC_EINVAL;
  int bit[3];
  for (int j = 0; j < k; ++j) bit[j] = nq - targets[j];
  int64_t N = (int64_t)1 << nq;
#pragma omp parallel for schedule(static)
  for (int64_t n = 0; n < N; ++n)
    out_amp(k, bit, U, in, (uint64_t)n, &out[2 * n], &out[2 * n + 1]);
  return ORC_OK;
}

/* Selected outputs only: out[2i], out[2i+1] = C~_{idx[i]}. */
int orc_apply_at(int nq, int k, const int *targets, const double *U,
                 const double *in, const uint64_t *idx, int64_t nidx,
                 double *out) {
  if (!check_targets(nq, k, targets) || !U || !in || !out || nidx < 0 ||
      (nidx > 0 && !idx))
    return ORC_EINVAL;
  int bit[3];
  for (int j = 0; j < k; ++j) bit[j] = nq - targets[j];
  uint64_t N = (uint64_t)1 << nq;
  for (int64_t i = 0; i < nidx; ++i)
    if (idx[i] >= N) return ORC_EINVAL;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < nidx; ++i)
    out_amp(k, bit, U, in, idx[i], &out[2 * i], &out[2 * i + 1]);
  return ORC_OK;
}

/* Same formula carried in long double, to bound the oracle's own rounding. */
int orc_apply_ld(int nq, int k, const int *targets, const double *U,
                 const double *in, double *out) {
  if (!check_targets(nq, k, targets) || !U || !in || !out || in == out)
    return ORC_EINVAL;
  int bit[3];
  for (int j = 0; j < k; ++j) bit[j] = nq - targets[j];
  int m = 1 << k;
  int64_t N = (int64_t)1 << nq;
#pragma omp parallel for schedule(static)
  for (int64_t n = 0; n < N; ++n) {
    int r = 0;
    for (int j = 0; j < k; ++j) r = (r << 1) | (int)(((uint64_t)n >> bit[j]) & 1u);
    uint64_t rest = (uint64_t)n;
    for (int j = 0; j < k; ++j) rest &= ~((uint64_t)1 << bit[j]);
    long double re = 0.0L, im = 0.0L;
    for (int c = 0; c < m; ++c) {
      uint64_t src = rest;
      for (int j = 0; j < k; ++j)
        if ((c >> (k - 1 - j)) & 1) src |= (uint64_t)1 << bit[j];
      long double ur = U[2 * (r * m + c)], ui = U[2 * (r * m + c) + 1];
      long double xr = in[2 * src], xi = in[2 * src + 1];
      re += ur * xr - ui * xi;
      im += ur * xi + ui * xr;
    }
    out[2 * n] = (double)re;
    out[2 * n + 1] = (double)im;
  }
  return ORC_OK;
}

/*
 * A circuit: gates applied in list order, i.e. the operator product read right
 * to left (CNOT_12 H_1 |00> applies H_1 first, §5 MV2-Noise description).
 * ks[g] is the gate size, targets[3g .. 3g+ks[g]-1] its targets and
 * mats + 2*mat_off[g] its matrix.  psi is updated; scratch holds 2^nq complex.
 */
int orc_circuit(int nq, int ngates, const int *ks, const int *targets,
                const double *mats, const int64_t *mat_off, double *psi,
                double *scratch) {
  if (ngates < 0 || !psi || !scratch || (ngates > 0 && (!ks || !targets || !mats || !mat_off)))
    return ORC_EINVAL;
  int64_t N = (int64_t)1 << nq;
  double *a = psi, *b = scratch;
  for (int g = 0; g < ngates; ++g) {
    int rc = orc_apply(nq, ks[g], targets + 3 * g, mats + 2 * mat_off[g], a, b);
    if (rc) return rc;
    double *t = a; a = b; b = t;
  }
  if (a != psi) memcpy(psi, a, (size_t)N * 2 * sizeof(double));
  return ORC_OK;
}

/* Many independent circuits (one per instance), instances spread over threads. */
int orc_circuit_batch(int ninst, const int *nqs, const int64_t *state_off,
                      const int *ngates, const int64_t *gate_off, const int *ks,
                      const int *targets, const double *mats,
                      const int64_t *mat_off, double *states) {
  if (ninst < 0) return ORC_EINVAL;
  int bad = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(| : bad)
  for (int i = 0; i < ninst; ++i) {
    int nq = nqs[i];
    if (nq < 1 || nq > 24) { bad |= 1; continue; }
    double *scratch = (double *)malloc(((size_t)1 << nq) * 2 * sizeof(double));
    if (!scratch) { bad |= 1; continue; }
    /* each instance runs single-threaded inside this thread */
    double *a = states + 2 * state_off[i], *b = scratch;
    int64_t N = (int64_t)1 << nq;
    for (int g = 0; g < ngates[i]; ++g) {
      int64_t gg = gate_off[i] + g;
      int k = ks[gg];
      const int *t = targets + 3 * gg;
      if (!check_targets(nq, k, t)) { bad |= 1; break; }
      int bit[3];
      for (int j = 0; j < k; ++j) bit[j] = nq - t[j];
      const double *U = mats + 2 * mat_off[gg];
      for (int64_t n = 0; n < N; ++n)
        out_amp(k, bit, U, a, (uint64_t)n, &b[2 * n], &b[2 * n + 1]);
      double *tmp = a; a = b; b = tmp;
    }
    if (a != states + 2 * state_off[i])
      memcpy(states + 2 * state_off[i], a, (size_t)N * 2 * sizeof(double));
    free(scratch);
  }
  return bad ? ORC_EINVAL : ORC_OK;
}

/*
 * Pick_k (§4a-§4c): the 2^nq / 2^k groups of labels that differ only in the
 * target qubits.  Found by scanning every label n in ascending order and
 * keeping those whose target qubits are all 0 (n_0 of Eq. pair0, n_00 of
 * Eq. twoopB); each such n contributes its m members in ascending local index
 * r, member r adding 2^(nq - is_j) for every target j whose value in r is 1
 * (n_1 = n_0 + 2^(nq - is), §3a; the quartet relations after Eq. resmat2).
 * out receives (2^nq / m) * m labels, group after group.
 */
int orc_pick(int nq, int k, const int *targets, uint64_t *out) {
  if (!check_targets(nq, k, targets) || !out || nq > 30) return ORC_EINVAL;
  int m = 1 << k;
  uint64_t stride[3];
  for (int j = 0; j < k; ++j) stride[j] = (uint64_t)1 << (nq - targets[j]);
  uint64_t N = (uint64_t)1 << nq, w = 0;
  for (uint64_t n = 0; n < N; ++n) {
    int zero = 1;
    for (int j = 0; j < k; ++j)
      if (n & stride[j]) zero = 0;
    if (!zero) continue;
    for (int r = 0; r < m; ++r) {
      uint64_t lab = n;
      for (int j = 0; j < k; ++j)
        if ((r >> (k - 1 - j)) & 1) lab += stride[j];
      out[w++] = lab;
    }
  }
  return ORC_OK;
}

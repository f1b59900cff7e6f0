// Gate fusion: runs of consecutive gates whose targets together span at most
// max_qubits qubits become one gate on that union.
//
// Gates compose in list order (the operator of a circuit is the product of
// its gates, the first gate rightmost), so a run g_1 .. g_r acting inside a
// qubit set Q is the single operator E(g_r) ... E(g_1) on Q, where E(g)
// extends g to Q by the identity on Q's other qubits (the tensor structure of
// §2c).  Only consecutive gates are merged; nothing is reordered.  The fused
// matrix carries the rounding of its products, so a fused circuit equals the
// original to rounding, not bit for bit.
#include <limits.h>
#include <string.h>

#include <complex>
#include <vector>

#include "qcw_host.h"

namespace qcw {

namespace {

using cd = std::complex<double>;

// A run being fused: its union of qubits and the product matrix on them
// (2^u x 2^u, row-major, u <= 3; fixed storage, no allocation).
struct Block {
  int u = 0;
  int q[3] = {0, 0, 0};  // union qubits, first = most significant local bit
  cd M[64];
};

int local_bit(const Block &b, int qubit) {
  for (int j = 0; j < b.u; ++j)
    if (b.q[j] == qubit) return b.u - 1 - j;
  return -1;
}

// Starts a block with one gate: its qubits in its own order, its matrix.
void start(Block &b, const qcw_gate &g, const qcw_c64 *U) {
  b.u = g.k;
  for (int j = 0; j < g.k; ++j) b.q[j] = g.q[j];
  const int mm = 1 << (2 * g.k);
  for (int e = 0; e < mm; ++e) b.M[e] = cd(U[e].re, U[e].im);
}

// Adds qubit `qubit` as the new least significant local bit: M <- M (x) I_2.
void grow(Block &b, int qubit) {
  const int m = 1 << b.u, m2 = 2 * m;
  cd M2[64];
  for (int e = 0; e < m2 * m2; ++e) M2[e] = cd(0.0, 0.0);
  for (int r = 0; r < m; ++r)
    for (int c = 0; c < m; ++c)
      for (int a = 0; a < 2; ++a) M2[(2 * r + a) * m2 + (2 * c + a)] = b.M[r * m + c];
  b.q[b.u++] = qubit;
  for (int e = 0; e < m2 * m2; ++e) b.M[e] = M2[e];
}

// M <- E(g) M, with E(g) the gate extended to the block's qubits.
void apply_gate(Block &b, const qcw_gate &g, const qcw_c64 *U) {
  const int m = 1 << b.u, mg = 1 << g.k;
  int bits[3];
  int mask = 0;
  for (int j = 0; j < g.k; ++j) {
    bits[j] = local_bit(b, g.q[j]);
    mask |= 1 << bits[j];
  }
  int spread[8];  // local index c of the gate -> block index bits
  for (int c = 0; c < mg; ++c) {
    int R = 0;
    for (int j = 0; j < g.k; ++j)
      if ((c >> (g.k - 1 - j)) & 1) R |= 1 << bits[j];
    spread[c] = R;
  }
  cd out[64];
  for (int R = 0; R < m; ++R) {
    const int rest = R & ~mask;
    int rg = 0;
    for (int j = 0; j < g.k; ++j) rg = (rg << 1) | ((R >> bits[j]) & 1);
    for (int C = 0; C < m; ++C) {
      // plain complex product (no Annex G special-case handling)
      double ar = 0.0, ai = 0.0;
      for (int c = 0; c < mg; ++c) {
        const qcw_c64 u = U[rg * mg + c];
        const cd v = b.M[(rest | spread[c]) * m + C];
        ar += u.re * v.real() - u.im * v.imag();
        ai += u.re * v.imag() + u.im * v.real();
      }
      out[R * m + C] = cd(ar, ai);
    }
  }
  for (int e = 0; e < m * m; ++e) b.M[e] = out[e];
}

}  // namespace

// Flops per amplitude of one k-qubit gate: m = 2^k outputs per group, each m
// complex products and m - 1 additions, per group of m amplitudes.
static int gate_flops(int k) { return 8 * (1 << k) - 2; }

int fuse_gate_list(const qcw_gate *gates, const int *idx, int n, const qcw_c64 *mats,
                   int max_qubits, int max_extra_flops, bool regroup,
                   std::vector<qcw_gate> *out_gates, std::vector<qcw_c64> *out_mats) {
  if (max_qubits < 1 || max_qubits > 3) return fail(QCW_EINVAL, "max_qubits=%d outside [1, 3]", max_qubits);
  out_gates->clear();
  out_mats->clear();
  out_gates->reserve((size_t)n);
  out_mats->reserve((size_t)64 * n);
  auto qmask = [](const qcw_gate &g) {
    uint64_t m = 0;
    for (int j = 0; j < g.k; ++j) m |= 1ull << g.q[j];
    return m;
  };
  // Emits one block: a lone gate as given (same bits as unfused), else the
  // product matrix on the block's qubits.
  auto emit = [&](const Block &b, const qcw_gate *lone) {
    qcw_gate g;
    memset(&g, 0, sizeof g);
    g.mat = (int64_t)out_mats->size();
    if (lone) {
      g.k = lone->k;
      for (int j = 0; j < lone->k; ++j) g.q[j] = lone->q[j];
      out_mats->insert(out_mats->end(), mats + lone->mat, mats + lone->mat + (1 << (2 * lone->k)));
    } else {
      g.k = b.u;
      for (int j = 0; j < b.u; ++j) g.q[j] = b.q[j];
      for (int e = 0; e < (1 << (2 * b.u)); ++e) out_mats->push_back({b.M[e].real(), b.M[e].imag()});
    }
    out_gates->push_back(g);
  };
  // Gates still to place, in order.  A block starts with the first of them
  // and scans the rest: a gate joins when the block stays within max_qubits
  // qubits and max_extra_flops, and (regroup) it shares no qubit with a gate
  // the scan has passed over -- such a gate commutes with everything it moves
  // ahead of.  Without regroup the scan stops at the first gate that cannot
  // join, so blocks are runs of consecutive gates.
  std::vector<int> rest(n), left;
  for (int i = 0; i < n; ++i) rest[i] = idx ? idx[i] : i;
  size_t head = 0;
  Block cur;
  while (head < rest.size()) {
    const qcw_gate &g0 = gates[rest[head]];
    start(cur, g0, mats + g0.mat);
    int members = 1;
    uint64_t skipped = 0;
    left.clear();
    size_t i = head + 1;
    for (; i < rest.size(); ++i) {
      const qcw_gate &g = gates[rest[i]];
      int fresh = 0;
      for (int j = 0; j < g.k; ++j) fresh += local_bit(cur, g.q[j]) < 0;
      const bool fits = !(qmask(g) & skipped) && cur.u + fresh <= max_qubits &&
                        gate_flops(cur.u + fresh) - gate_flops(cur.u) - gate_flops(g.k) <=
                            max_extra_flops;
      if (fits) {
        for (int j = 0; j < g.k; ++j)
          if (local_bit(cur, g.q[j]) < 0) grow(cur, g.q[j]);
        apply_gate(cur, g, mats + g.mat);
        ++members;
      } else if (regroup) {
        skipped |= qmask(g);
        left.push_back(rest[i]);
      } else {
        break;
      }
    }
    emit(cur, members == 1 ? &g0 : nullptr);
    if (regroup) {
      rest.swap(left);
      head = 0;
    } else {
      head = i;
    }
  }
  return QCW_OK;
}

int fuse_circuit(int nq, const qcw_gate *gates, int ngates, const qcw_c64 *mats, int64_t nmats,
                 int max_qubits, bool regroup, std::vector<qcw_gate> *out_gates,
                 std::vector<qcw_c64> *out_mats) {
  for (int i = 0; i < ngates; ++i) {
    const qcw_gate &g = gates[i];
    Geom geo;
    int rc = make_geom(nq, g.k, g.q, &geo);
    if (rc) return rc;
    if (g.mat < 0 || g.mat + ((int64_t)1 << (2 * g.k)) > nmats)
      return fail(QCW_EINVAL, "gate %d: matrix offset outside mats", i);
  }
  return fuse_gate_list(gates, nullptr, ngates, mats, max_qubits, INT_MAX, regroup, out_gates,
                        out_mats);
}

}  // namespace qcw

using namespace qcw;

extern "C" int qcw_fuse_circuit(int nq, const qcw_gate *gates, int ngates, const qcw_c64 *mats,
                                int64_t nmats, int max_qubits, int regroup, qcw_gate *out_gates,
                                int *out_ngates, qcw_c64 *out_mats, int64_t out_mats_cap,
                                int64_t *out_nmats) {
  clear_error();
  if (nq < 1 || nq > kMaxQubits) return fail(QCW_EINVAL, "nq=%d outside [1, %d]", nq, kMaxQubits);
  if (ngates < 0 || (ngates > 0 && (!gates || !mats)) || !out_ngates || !out_nmats ||
      (ngates > 0 && !out_gates))
    return fail(QCW_EINVAL, "NULL argument");
  std::vector<qcw_gate> g;
  std::vector<qcw_c64> m;
  if (regroup != 0 && regroup != 1) return fail(QCW_EINVAL, "regroup=%d is not 0 or 1", regroup);
  int rc = fuse_circuit(nq, gates, ngates, mats, nmats, max_qubits, regroup != 0, &g, &m);
  if (rc) return rc;
  if ((int64_t)m.size() > out_mats_cap || (!m.empty() && !out_mats))
    return fail(QCW_EINVAL, "out_mats holds %lld entries, %zu needed", (long long)out_mats_cap,
                m.size());
  if (!g.empty()) memcpy(out_gates, g.data(), g.size() * sizeof(qcw_gate));
  if (!m.empty()) memcpy(out_mats, m.data(), m.size() * sizeof(qcw_c64));
  *out_ngates = (int)g.size();
  *out_nmats = (int64_t)m.size();
  return QCW_OK;
}

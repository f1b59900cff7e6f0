// Host side of the batched form: validation, work-item planning (largest
// instances first), the per-qubit-count tile-shape table, hipGraph capture of
// the persistent launch, and the autotuner that writes the table.
#include <hip/hip_runtime.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <map>
#include <numeric>
#include <string>
#include <vector>

#include "qcw_batch.h"

namespace qcw {

static const char *kVarNames[kVarCount] = {"amp4_sgpr", "amp8_sgpr", "amp16_sgpr",
                                           "amp4_lds", "amp8_lds", "amp4_mfma"};

const char *variant_name(int v) { return (v >= 0 && v < kVarCount) ? kVarNames[v] : "?"; }

int variant_from_name(const char *s) {
  for (int v = 0; v < kVarCount; ++v)
    if (!strcmp(s, kVarNames[v])) return v;
  return -1;
}

void tune_defaults(TuneTable *t) {
  for (int nq = 0; nq <= kBatchMaxNq; ++nq)
    t->variant[nq] = nq <= 6 ? kVarAmp4Sgpr : kVarAmp8Sgpr;
  t->from_file = false;
}

static std::string device_arch() {
  int dev = 0;
  hipDeviceProp_t p;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&p, dev) != hipSuccess) {
    (void)hipGetLastError();
    return "unknown";
  }
  std::string a = p.gcnArchName;
  size_t colon = a.find(':');
  return colon == std::string::npos ? a : a.substr(0, colon);
}

int tune_load(const char *path, TuneTable *t) {
  tune_defaults(t);
  if (!path || !*path) return QCW_OK;
  FILE *f = fopen(path, "r");
  if (!f) return fail(QCW_EINVAL, "cannot open tune table %s", path);
  char line[256];
  std::string arch;
  int rc = QCW_OK;
  while (fgets(line, sizeof line, f)) {
    if (line[0] == '#' || line[0] == '\n') continue;
    char key[32] = {0}, name[32] = {0};
    int nq = 0;
    if (sscanf(line, "arch %31s", key) == 1) {
      arch = key;
    } else if (sscanf(line, "nq %d variant %31s", &nq, name) == 2) {
      int v = variant_from_name(name);
      if (nq < 1 || nq > kBatchMaxNq || v < 0) {
        rc = fail(QCW_EINVAL, "tune table %s: bad line '%s'", path, line);
        break;
      }
      t->variant[nq] = v;
    }
  }
  fclose(f);
  if (rc) return rc;
  if (arch != device_arch())
    return fail(QCW_EINVAL, "tune table %s is for %s, device is %s", path, arch.c_str(),
                device_arch().c_str());
  t->from_file = true;
  return QCW_OK;
}

int make_bgate(int nq, const qcw_gate &g, int64_t nmats, BGate *out) {
  Geom geo;
  int rc = make_geom(nq, g.k, g.q, &geo);
  if (rc) return rc;
  const int64_t mm = (int64_t)1 << (2 * g.k);
  if (g.mat < 0 || g.mat + mm > nmats) return fail(QCW_EINVAL, "matrix offset outside mats");
  memset(out, 0, sizeof *out);
  out->k = g.k;
  out->sb0 = geo.sb[0];
  out->sb1 = geo.sb[1];
  out->sb2 = geo.sb[2];
  for (int r = 0; r < 8; ++r) out->off[r] = (uint32_t)geo.off[r];
  out->mat_off = g.mat;
  return QCW_OK;
}

// Grid of one persistent kernel: each wave needs per_wave bytes of LDS; a
// block holds as many waves (up to four) as fit in 64 KiB of dynamic LDS.
static int plan_shape(int max_nq, int nitems, size_t per_wave, bool mfma, BatchShape *sh) {
  *sh = BatchShape{};
  if (nitems <= 0) return QCW_OK;
  if (per_wave > 64 * 1024) return fail(QCW_EINVAL, "instances of %d qubits exceed LDS", max_nq);
  const int wpb = (int)std::max<size_t>(1, std::min<size_t>(kBatchBlock / 64, (64 * 1024) / per_wave));
  const size_t lds = per_wave * wpb;
  int bpc = 0;
  int rc = mfma ? batch_mfma_occupancy(lds, wpb * 64, &bpc) : batch_kernel_occupancy(lds, wpb * 64, &bpc);
  if (rc) return rc;
  if (bpc < 1) return fail(QCW_EINVAL, "batch kernel does not fit a CU with %zu B of LDS", lds);
  int dev = 0, ncu = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
    (void)hipGetLastError();
    return fail(QCW_EHIP, "cannot query the device");
  }
  const int blocks_needed = (nitems + wpb - 1) / wpb;
  sh->wave_amps = 1 << std::max(max_nq, 1);
  sh->lds_bytes = lds;
  sh->threads = wpb * 64;
  sh->blocks = (unsigned)std::max(1, std::min(ncu * bpc, blocks_needed));
  return QCW_OK;
}

int plan_batch_launch(int max_nq, int n_exact, int n_mfma, BatchLaunch *L) {
  const size_t amps = (size_t)1 << std::max(max_nq, 1);
  // exact kernel: state plus two 64-entry matrix slots; matrix-core kernel: state only
  int rc = plan_shape(max_nq, n_exact, (amps + 128) * sizeof(double2), false, &L->ex);
  if (rc) return rc;
  return plan_shape(max_nq, n_mfma, amps * sizeof(double2), true, &L->mf);
}

// Deals one persistent kernel's items (sorted largest first) to its blocks so
// that the blocks resident together on a CU mix large and small items.  The
// dispatcher places blocks on CUs in index order, one round over all CUs at a
// time, so residency slot j of the CUs holds blocks [j * ncu, (j + 1) * ncu);
// in every other slot the groups of items are dealt in reverse, which pairs
// the largest items of one slot with the smallest of the next.  Applies only
// when every item has its own wave and the items fill whole blocks (the item
// index of a wave is then its block's index times waves per block plus its
// wave), so no wave is left without an item in the middle of the list.
void snake_items(BItem *items, int n, const BatchShape &sh, int ncu) {
  const int wpb = sh.threads / 64;
  if (n <= 0 || wpb < 1 || n % wpb || (int64_t)n > (int64_t)sh.blocks * wpb || ncu < 1) return;
  const int nb = n / wpb;
  if (nb <= ncu) return;
  std::vector<BItem> src(items, items + n);
  for (int i = 0; i < nb; ++i) {
    const int j = i / ncu, p = i % ncu;
    const int in_slot = std::min(ncu, nb - j * ncu);
    const int blk = (j & 1) ? j * ncu + (in_slot - 1 - p) : i;
    for (int w = 0; w < wpb; ++w) items[blk * wpb + w] = src[i * wpb + w];
  }
}

// Largest batch-resident instance: each wave needs (2^nq + 128) * 16 bytes of
// LDS, 34 KiB at nq = 11.  Larger instances run as plain sweeps in the same graph.
constexpr int kBatchResidentNq = 11;
// Most executions one graph of qcw_batch_run_repeat may hold.
constexpr int kBatchMaxRepeat = 1024;

}  // namespace qcw

using namespace qcw;

struct qcw_batch {
  int n = 0;
  qcw_c64 *states = nullptr;
  BGate *gates_d = nullptr;
  double2 *mats_d = nullptr;
  BItem *items_d = nullptr;
  int *counter_d = nullptr;
  BatchLaunch L{};
  int nitems = 0;
  std::vector<BInst> inst_h;
  std::vector<qcw_gate> gates_h;
  std::vector<qcw_c64> mats_h;
  std::vector<int> big;  // instances run as plain sweeps
  TuneTable tune;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  // graphs of several executions in a row (qcw_batch_run_repeat), per count
  std::map<int, std::pair<hipGraph_t, hipGraphExec_t>> repeat;
};

static void batch_free(qcw_batch *b) {
  if (!b) return;
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  for (auto &r : b->repeat) {
    if (r.second.second) (void)hipGraphExecDestroy(r.second.second);
    if (r.second.first) (void)hipGraphDestroy(r.second.first);
  }
  (void)hipFree(b->gates_d);
  (void)hipFree(b->mats_d);
  (void)hipFree(b->items_d);
  (void)hipFree(b->counter_d);
  delete b;
}

template <typename T>
static int upload(T **dst, const T *src, size_t n, const char *what) {
  size_t bytes = std::max<size_t>(n, 1) * sizeof(T);
  if (hipMalloc((void **)dst, bytes) != hipSuccess) {
    (void)hipGetLastError();
    return fail(QCW_ENOMEM, "hipMalloc for %s (%zu B) failed", what, bytes);
  }
  if (n && hipMemcpy(*dst, src, n * sizeof(T), hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipGetLastError();
    return fail(QCW_EHIP, "upload of %s failed", what);
  }
  return QCW_OK;
}

// Enqueues one execution of the batch (persistent launch + oversize instances).
static int enqueue_batch(qcw_batch *b, hipStream_t s) {
  int rc = launch_batch(b->L, s);
  if (rc) return rc;
  for (int i : b->big) {
    const BInst &in = b->inst_h[i];
    for (int g = 0; g < in.ngates; ++g) {
      const qcw_gate &gt = b->gates_h[in.gate_off + g];
      Geom geo;
      if ((rc = make_geom(in.nq, gt.k, gt.q, &geo))) return rc;
      qcw_c64 *psi = b->states + in.state_off;
      if ((rc = launch_sweep(geo, b->mats_h.data() + gt.mat, psi, psi, s))) return rc;
    }
  }
  return QCW_OK;
}

static int batch_build(qcw_batch *b, const qcw_instance *inst, int n, const qcw_gate *gates,
                       int64_t ngates, const qcw_c64 *mats, int64_t nmats, qcw_c64 *states,
                       int64_t nstates, const int *variant_override) {
  b->n = n;
  b->states = states;
  b->gates_h.assign(gates, gates + ngates);
  b->mats_h.assign(mats, mats + nmats);
  std::vector<BGate> bg((size_t)ngates);
  std::vector<char> gate_nq_checked((size_t)ngates, 0);
  b->inst_h.resize(n);
  std::vector<std::pair<int64_t, int64_t>> ranges;
  int max_nq = 1;
  for (int i = 0; i < n; ++i) {
    const qcw_instance &q = inst[i];
    if (q.nq < 1 || q.nq > kMaxQubits) return fail(QCW_EINVAL, "instance %d: nq=%d", i, q.nq);
    if (q.ngates < 0 || q.gate_off < 0 || q.gate_off + q.ngates > ngates)
      return fail(QCW_EINVAL, "instance %d: gate range outside gates", i);
    const int64_t N = (int64_t)1 << q.nq;
    if (q.state_off < 0 || q.state_off + N > nstates)
      return fail(QCW_EINVAL, "instance %d: state outside the states buffer", i);
    ranges.push_back({q.state_off, q.state_off + N});
    for (int g = 0; g < q.ngates; ++g) {
      BGate tmp;
      int rc = make_bgate(q.nq, gates[q.gate_off + g], nmats, &tmp);
      if (rc) {
        char why[400];
        snprintf(why, sizeof why, "%s", qcw_last_error());
        return fail(rc, "instance %d gate %d: %s", i, g, why);
      }
      // A gate shared by instances of different sizes gets the geometry of
      // each user; sharing is only allowed between instances of equal nq.
      if (gate_nq_checked[q.gate_off + g] && gate_nq_checked[q.gate_off + g] != q.nq)
        return fail(QCW_EINVAL, "gate %lld is shared by instances of different nq",
                    (long long)(q.gate_off + g));
      gate_nq_checked[q.gate_off + g] = (char)q.nq;
      bg[q.gate_off + g] = tmp;
    }
    b->inst_h[i] = {q.nq, q.ngates, q.state_off, q.gate_off};
    if (q.nq <= kBatchResidentNq) max_nq = std::max(max_nq, q.nq);
  }
  std::sort(ranges.begin(), ranges.end());
  for (size_t i = 1; i < ranges.size(); ++i)
    if (ranges[i].first < ranges[i - 1].second)
      return fail(QCW_EINVAL, "instance states overlap");

  // Work items: LDS-resident instances, most work first.
  std::vector<BItem> items;
  std::vector<int> item_inst;  // instance of each item
  for (int i = 0; i < n; ++i) {
    const BInst &in = b->inst_h[i];
    if (in.nq > kBatchResidentNq) {
      b->big.push_back(i);
      continue;
    }
    int v = variant_override ? variant_override[in.nq] : b->tune.variant[in.nq];
    items.push_back({in.nq, v, 0, in.ngates, in.state_off, in.gate_off,
                     in.ngates > 0 ? gates[in.gate_off].mat : 0,
                     in.ngates > 1 ? gates[in.gate_off + 1].mat : 0,
                     in.ngates > 0 ? gates[in.gate_off].k : 0,
                     in.ngates > 1 ? gates[in.gate_off + 1].k : 0, {0, 0}});
    item_inst.push_back(i);
  }
  // Instances on the matrix-core variant (already exact only to rounding) run
  // their circuits fused into gates of at most three qubits.  Instances that
  // share a gate range share its fused copy.
  std::vector<double2> m2((size_t)nmats);
  for (int64_t i = 0; i < nmats; ++i) m2[i] = make_double2(mats[i].re, mats[i].im);
  std::map<std::pair<int64_t, int>, std::pair<int64_t, int>> fused_at;
  for (size_t ii = 0; ii < items.size(); ++ii) {
    BItem &it = items[ii];
    if (it.variant != kVarAmp4Mfma) continue;
    BInst &in = b->inst_h[item_inst[ii]];
    auto key = std::make_pair(in.gate_off, in.ngates);
    auto f = fused_at.find(key);
    if (f == fused_at.end()) {
      std::vector<qcw_gate> fg;
      std::vector<qcw_c64> fm;
      int rc = fuse_circuit(in.nq, gates + in.gate_off, in.ngates, mats, nmats,
                            std::min(3, in.nq), true, &fg, &fm);
      if (rc) return rc;
      const int64_t goff = (int64_t)bg.size(), moff = (int64_t)m2.size();
      for (const qcw_c64 &z : fm) m2.push_back(make_double2(z.re, z.im));
      for (qcw_gate g : fg) {
        BGate t;
        g.mat += moff;
        if ((rc = make_bgate(in.nq, g, (int64_t)m2.size(), &t))) return rc;
        bg.push_back(t);
      }
      f = fused_at.emplace(key, std::make_pair(goff, (int)fg.size())).first;
    }
    in.gate_off = f->second.first;
    in.ngates = f->second.second;
    it.gate_off = in.gate_off;
    it.g_end = in.ngates;
  }
  // the first two gates' matrices, for the matrix-core kernel (offsets into m2)
  for (BItem &it : items) {
    if (it.variant != kVarAmp4Mfma || it.g_end <= it.g_begin) continue;
    const BGate &g0 = bg[it.gate_off + it.g_begin];
    it.mat0 = g0.mat_off;
    it.k0 = g0.k;
    if (it.g_end - it.g_begin > 1) {
      const BGate &g1 = bg[it.gate_off + it.g_begin + 1];
      it.mat1 = g1.mat_off;
      it.k1 = g1.k;
    }
  }
  // Exact-kernel items first, then matrix-core items; most work first in each.
  std::stable_sort(items.begin(), items.end(), [&](const BItem &x, const BItem &y) {
    const bool mx = x.variant == kVarAmp4Mfma, my = y.variant == kVarAmp4Mfma;
    if (mx != my) return my;
    return ((int64_t)(x.g_end - x.g_begin) << x.nq) > ((int64_t)(y.g_end - y.g_begin) << y.nq);
  });
  b->nitems = (int)items.size();
  int n_exact = 0;
  for (const BItem &it : items) n_exact += it.variant != kVarAmp4Mfma;

  // Grids first, so the items can be dealt to their blocks.
  int rc = plan_batch_launch(max_nq, n_exact, b->nitems - n_exact, &b->L);
  if (rc) return rc;
  {
    int dev = 0, ncu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
      (void)hipGetLastError();
      return fail(QCW_EHIP, "cannot query the device");
    }
    snake_items(items.data(), n_exact, b->L.ex, ncu);
    snake_items(items.data() + n_exact, b->nitems - n_exact, b->L.mf, ncu);
  }
  if ((rc = upload(&b->gates_d, bg.data(), bg.size(), "gates"))) return rc;
  if ((rc = upload(&b->mats_d, m2.data(), m2.size(), "matrices"))) return rc;
  if ((rc = upload(&b->items_d, items.data(), items.size(), "work items"))) return rc;
  const int zeros[2] = {0, 0};
  if ((rc = upload(&b->counter_d, zeros, 2, "work counters"))) return rc;

  b->L.items = b->items_d;
  b->L.nitems = b->nitems;
  b->L.n_exact = n_exact;
  b->L.gates = b->gates_d;
  b->L.mats = b->mats_d;
  b->L.states = reinterpret_cast<double2 *>(states);
  b->L.counter = b->counter_d;
  return QCW_OK;
}

// Captures `reps` executions of the batch, one after another, into a graph
// on `user` (NULL: a private stream) and instantiates it.
static int capture(qcw_batch *b, hipStream_t user, int reps, hipGraph_t *graph,
                   hipGraphExec_t *exec) {
  hipStream_t s = user;
  bool own = false;
  if (!s) {
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
      (void)hipGetLastError();
      return fail(QCW_EHIP, "cannot create a capture stream");
    }
    own = true;
  }
  int rc = QCW_OK;
  const bool timing = timing_on();
  if (timing) qcw_timing_enable(0);
  if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    (void)hipGetLastError();
    rc = fail(QCW_EHIP, "hipStreamBeginCapture failed");
  } else {
    for (int r = 0; r < reps && !rc; ++r) rc = enqueue_batch(b, s);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(s, &g);
    if (!rc && e != hipSuccess) rc = fail(QCW_EHIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
    *graph = g;
    if (!rc && hipGraphInstantiate(exec, g, nullptr, nullptr, 0) != hipSuccess) {
      (void)hipGetLastError();
      rc = fail(QCW_EHIP, "hipGraphInstantiate failed");
    }
  }
  if (timing) qcw_timing_enable(1);
  if (own) (void)hipStreamDestroy(s);
  return rc;
}

extern "C" {

int qcw_batch_create(qcw_batch **out, const qcw_instance *inst, int n, const qcw_gate *gates,
                     int64_t ngates, const qcw_c64 *mats, int64_t nmats, qcw_c64 *states,
                     int64_t nstates, const char *tune_table, void *stream) {
  clear_error();
  if (!out) return fail(QCW_EINVAL, "out is NULL");
  *out = nullptr;
  if (n < 0 || ngates < 0 || nmats < 0 || nstates < 0) return fail(QCW_EINVAL, "negative count");
  if ((n > 0 && !inst) || (ngates > 0 && !gates) || (nmats > 0 && !mats))
    return fail(QCW_EINVAL, "NULL input array");
  if (n > 0) {
    int rc = check_device_range(states, (uint64_t)nstates * sizeof(qcw_c64), "states");
    if (rc) return rc;
  }
  qcw_batch *b = new qcw_batch();
  int rc = tune_load(tune_table, &b->tune);
  if (!rc) rc = batch_build(b, inst, n, gates, ngates, mats, nmats, states, nstates, nullptr);
  if (!rc) rc = capture(b, (hipStream_t)stream, 1, &b->graph, &b->exec);
  if (rc) {
    batch_free(b);
    return rc;
  }
  *out = b;
  return QCW_OK;
}

int qcw_batch_run(qcw_batch *b, void *stream) {
  clear_error();
  if (!b || !b->exec) return fail(QCW_EINVAL, "invalid batch handle");
  TimedLaunch t(kKernelBatch, (hipStream_t)stream);
  hipError_t e = hipGraphLaunch(b->exec, (hipStream_t)stream);
  if (e != hipSuccess) return fail(QCW_EHIP, "hipGraphLaunch: %s", hipGetErrorString(e));
  return QCW_OK;
}

int qcw_batch_run_repeat(qcw_batch *b, int reps, void *stream) {
  clear_error();
  if (!b || !b->exec) return fail(QCW_EINVAL, "invalid batch handle");
  if (reps < 1 || reps > kBatchMaxRepeat)
    return fail(QCW_EINVAL, "reps=%d outside [1, %d]", reps, kBatchMaxRepeat);
  if (reps == 1) return qcw_batch_run(b, stream);
  auto it = b->repeat.find(reps);
  if (it == b->repeat.end()) {
    hipGraph_t g = nullptr;
    hipGraphExec_t x = nullptr;
    int rc = capture(b, nullptr, reps, &g, &x);
    if (rc) {
      if (x) (void)hipGraphExecDestroy(x);
      if (g) (void)hipGraphDestroy(g);
      return rc;
    }
    it = b->repeat.emplace(reps, std::make_pair(g, x)).first;
  }
  TimedLaunch t(kKernelBatch, (hipStream_t)stream);
  hipError_t e = hipGraphLaunch(it->second.second, (hipStream_t)stream);
  if (e != hipSuccess) return fail(QCW_EHIP, "hipGraphLaunch: %s", hipGetErrorString(e));
  return QCW_OK;
}

int qcw_batch_run_eager(qcw_batch *b, void *stream) {
  clear_error();
  if (!b) return fail(QCW_EINVAL, "invalid batch handle");
  return enqueue_batch(b, (hipStream_t)stream);
}

int qcw_batch_info(const qcw_batch *b, int nq, int *variant, int *blocks, int *lds_bytes) {
  clear_error();
  if (!b) return fail(QCW_EINVAL, "invalid batch handle");
  if (variant) *variant = (nq >= 1 && nq <= kBatchMaxNq) ? b->tune.variant[nq] : -1;
  const int v = (nq >= 1 && nq <= kBatchMaxNq) ? b->tune.variant[nq] : -1;
  const BatchShape &sh = (v == kVarAmp4Mfma && b->L.mf.blocks) || !b->L.ex.blocks ? b->L.mf : b->L.ex;
  if (blocks) *blocks = (int)sh.blocks;
  if (lds_bytes) *lds_bytes = (int)sh.lds_bytes;
  return QCW_OK;
}

int qcw_batch_destroy(qcw_batch *b) {
  clear_error();
  batch_free(b);
  return QCW_OK;
}

const char *qcw_batch_variant_name(int v) { return variant_name(v); }

}  // extern "C"

// ------------------------------------------------------------------ autotuner
namespace {

struct SplitMix {
  uint64_t s;
  uint64_t next() {
    uint64_t z = (s += 0x9e3779b97f4a7c15ULL);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
  }
  double uni() { return (double)(next() >> 11) * (1.0 / 9007199254740992.0) * 2.0 - 1.0; }
  int below(int n) { return (int)(next() % (uint64_t)n); }
};

// A unitary m x m matrix: Gram-Schmidt over the columns of a random matrix.
void random_unitary(SplitMix &r, int m, qcw_c64 *U) {
  std::vector<std::complex<double>> a((size_t)m * m);
  for (auto &z : a) z = {r.uni(), r.uni()};
  for (int j = 0; j < m; ++j) {
    for (int i = 0; i < j; ++i) {
      std::complex<double> d = 0;
      for (int t = 0; t < m; ++t) d += std::conj(a[t * m + i]) * a[t * m + j];
      for (int t = 0; t < m; ++t) a[t * m + j] -= d * a[t * m + i];
    }
    double nrm = 0;
    for (int t = 0; t < m; ++t) nrm += std::norm(a[t * m + j]);
    nrm = std::sqrt(nrm);
    for (int t = 0; t < m; ++t) a[t * m + j] /= nrm;
  }
  for (int i = 0; i < m * m; ++i) U[i] = {a[i].real(), a[i].imag()};
}

}  // namespace

extern "C" int qcw_batch_autotune(const char *out_path, int nq_lo, int nq_hi, int ninst,
                                  int gates_per_qubit, void *stream) {
  clear_error();
  if (!out_path) return fail(QCW_EINVAL, "out_path is NULL");
  if (nq_lo < 1 || nq_hi > kBatchResidentNq || nq_lo > nq_hi)
    return fail(QCW_EINVAL, "qubit range must lie in [1, %d]", kBatchResidentNq);
  if (ninst < 1 || gates_per_qubit < 1) return fail(QCW_EINVAL, "ninst and gates_per_qubit >= 1");
  hipStream_t s = (hipStream_t)stream;
  TuneTable best;
  tune_defaults(&best);
  std::string report;
  SplitMix rng{0x5eed};
  for (int nq = nq_lo; nq <= nq_hi; ++nq) {
    const int G = gates_per_qubit * nq;
    std::vector<qcw_instance> inst(ninst);
    std::vector<qcw_gate> gates;
    std::vector<qcw_c64> mats;
    for (int i = 0; i < ninst; ++i) {
      inst[i] = {nq, G, (int64_t)i << nq, (int64_t)gates.size()};
      for (int g = 0; g < G; ++g) {
        int u = rng.below(100);
        int k = u < 50 ? 1 : (u < 85 ? 2 : 3);
        k = std::min(k, nq);
        qcw_gate gt{};
        gt.k = k;
        for (int j = 0; j < k; ++j) {
          int t;
          bool dup;
          do {
            t = 1 + rng.below(nq);
            dup = false;
            for (int q = 0; q < j; ++q) dup |= gt.q[q] == t;
          } while (dup);
          gt.q[j] = t;
        }
        gt.mat = (int64_t)mats.size();
        mats.resize(mats.size() + ((size_t)1 << (2 * k)));
        random_unitary(rng, 1 << k, mats.data() + gt.mat);
        gates.push_back(gt);
      }
    }
    const int64_t nstates = (int64_t)ninst << nq;
    qcw_c64 *states = nullptr;
    hipError_t he = hipMalloc(&states, (size_t)nstates * sizeof(qcw_c64));
    if (he != hipSuccess) {
      (void)hipGetLastError();
      return fail(he == hipErrorOutOfMemory ? QCW_ENOMEM : QCW_EHIP,
                  "autotune nq=%d: hipMalloc(%lld B): %s", nq,
                  (long long)(nstates * (int64_t)sizeof(qcw_c64)), hipGetErrorString(he));
    }
    std::vector<qcw_c64> psi((size_t)nstates);
    const double amp = 1.0 / std::sqrt((double)(1 << nq));
    for (auto &z : psi) z = {amp, 0.0};
    he = hipMemcpy(states, psi.data(), psi.size() * sizeof(qcw_c64), hipMemcpyHostToDevice);
    if (he != hipSuccess) {
      (void)hipFree(states);
      return fail(QCW_EHIP, "autotune nq=%d: upload: %s", nq, hipGetErrorString(he));
    }
    float best_ms = 1e30f;
    char line[256];
    std::string times;
    for (int v = 0; v < kVarCount; ++v) {
      int ov[kBatchMaxNq + 1];
      for (int q = 0; q <= kBatchMaxNq; ++q) ov[q] = v;
      qcw_batch *b = new qcw_batch();
      tune_defaults(&b->tune);
      int rc = batch_build(b, inst.data(), ninst, gates.data(), (int64_t)gates.size(),
                           mats.data(), (int64_t)mats.size(), states, nstates, ov);
      if (rc) {
        batch_free(b);
        (void)hipFree(states);
        return rc;
      }
      hipEvent_t e0, e1;
      (void)hipEventCreate(&e0);
      (void)hipEventCreate(&e1);
      float ms_min = 1e30f;
      for (int rep = 0; rep < 6; ++rep) {
        (void)hipEventRecord(e0, s);
        rc = launch_batch(b->L, s);
        (void)hipEventRecord(e1, s);
        if (rc) break;
        hipError_t ee = hipEventSynchronize(e1);
        float ms = 0;
        if (ee == hipSuccess) ee = hipEventElapsedTime(&ms, e0, e1);
        if (ee != hipSuccess) {
          rc = fail(QCW_EHIP, "autotune nq=%d variant %s: %s", nq, variant_name(v),
                    hipGetErrorString(ee));
          break;
        }
        if (rep > 0) ms_min = std::min(ms_min, ms);
      }
      (void)hipEventDestroy(e0);
      (void)hipEventDestroy(e1);
      batch_free(b);
      if (rc) {
        (void)hipFree(states);
        return rc;
      }
      snprintf(line, sizeof line, " %s=%.1f", variant_name(v), ms_min * 1000.0f);
      times += line;
      if (ms_min < best_ms) {
        best_ms = ms_min;
        best.variant[nq] = v;
      }
    }
    (void)hipFree(states);
    snprintf(line, sizeof line, "nq %d variant %s us %.1f # instances %d gates %d;%s\n", nq,
             variant_name(best.variant[nq]), best_ms * 1000.0f, ninst, G, times.c_str());
    report += line;
  }
  FILE *f = fopen(out_path, "w");
  if (!f) return fail(QCW_EINVAL, "cannot write %s", out_path);
  fprintf(f, "# qcw batch tune table: fastest tile shape per qubit count (times in us,\n");
  fprintf(f, "# one persistent launch over the listed synthetic batch)\n");
  fprintf(f, "arch %s\n", device_arch().c_str());
  fputs(report.c_str(), f);
  fclose(f);
  return QCW_OK;
}

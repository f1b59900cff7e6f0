// GPU executor of the continuous-batching request loop and its C ABI.
//
// Device memory: one arena of the configured budget.  An admitted request
// occupies [state | gate table | matrices] at its arena offset until it
// completes, so its state stays resident across ticks.  A tick uploads the
// small instance and work-item tables of the resident requests (pinned host
// buffers, async copies), runs ONE persistent batch launch (the same kernel
// as qcw_batch_run) over them, copies the states of finishing requests to
// pinned host buffers and waits for the tick's event.
#include <hip/hip_runtime.h>
#include <string.h>

#include <algorithm>
#include <memory>
#include <vector>

#include "qcw_batch.h"
#include "server_core.h"

namespace qcw {

namespace {

uint64_t round256(uint64_t x) { return (x + 255) & ~uint64_t(255); }

class HipExecutor : public Executor {
 public:
  ~HipExecutor() override {
    if (stream_) (void)hipStreamSynchronize(stream_);
    (void)hipFree(arena_);
    (void)hipFree(inst_d_);
    (void)hipFree(items_d_);
    (void)hipFree(counter_d_);
    (void)hipHostFree(inst_h_);
    (void)hipHostFree(items_h_);
    (void)hipHostFree(result_h_);
    if (done_) (void)hipEventDestroy(done_);
    if (stream_) (void)hipStreamDestroy(stream_);
  }

  int init(const ServerConfig &cfg, const char *tune_table) {
    if (hipGetDevice(&dev_) != hipSuccess) return hip_fail("hipGetDevice");
    max_slots_ = cfg.max_slots;
    max_nq_ = cfg.max_nq;
    int rc = tune_load(tune_table, &tune_);
    if (rc) return rc;
    if (hipStreamCreateWithFlags(&stream_, hipStreamNonBlocking) != hipSuccess)
      return hip_fail("stream");
    if (hipEventCreateWithFlags(&done_, hipEventDisableTiming) != hipSuccess)
      return hip_fail("event");
    arena_bytes_ = cfg.hbm_budget_bytes & ~uint64_t(255);
    if (hipMalloc(&arena_, std::max<uint64_t>(arena_bytes_, 256)) != hipSuccess)
      return mem_fail("arena", arena_bytes_);
    if (hipMalloc(&inst_d_, sizeof(BInst) * max_slots_) != hipSuccess ||
        hipMalloc(&items_d_, sizeof(BItem) * max_slots_) != hipSuccess ||
        hipMalloc(&counter_d_, 2 * sizeof(int)) != hipSuccess)
      return mem_fail("tables", 0);
    if (hipHostMalloc(&inst_h_, sizeof(BInst) * max_slots_) != hipSuccess ||
        hipHostMalloc(&items_h_, sizeof(BItem) * max_slots_) != hipSuccess ||
        hipHostMalloc(&result_h_, sizeof(qcw_c64) * ((size_t)max_slots_ << max_nq_)) != hipSuccess)
      return mem_fail("pinned host buffers", 0);
    slots_.resize(max_slots_);
    return QCW_OK;
  }

  // Requests whose size runs on the matrix-core variant are fused into gates
  // of at most three qubits, as in the batched form.
  int prepare(ServeRequest *r) override {
    if (r->ngates == 0 || tune_.variant[r->nq] != kVarAmp4Mfma) return QCW_OK;
    std::vector<qcw_gate> fg;
    std::vector<qcw_c64> fm;
    int rc = fuse_circuit(r->nq, r->gates.data(), r->ngates, r->mats.data(),
                          (int64_t)r->mats.size(), std::min(3, r->nq), true, &fg, &fm);
    if (rc) return rc;
    r->gates.swap(fg);
    r->mats.swap(fm);
    r->ngates = (int)r->gates.size();
    return QCW_OK;
  }

  int load(int slot, uint64_t off, const ServeRequest &r) override {
    (void)hipSetDevice(dev_);
    SlotInfo &s = slots_[slot];
    const uint64_t sbytes = round256((uint64_t)16 << r.nq);
    const uint64_t gbytes = round256((uint64_t)64 * r.ngates);
    s.nq = r.nq;
    s.ngates = r.ngates;
    s.state_off = (int64_t)(off / 16);
    s.gate_off = (int64_t)((off + sbytes) / 64);
    const int64_t mat_base = (int64_t)((off + sbytes + gbytes) / 16);
    std::vector<BGate> bg(r.ngates);
    for (int g = 0; g < r.ngates; ++g) {
      int rc = make_bgate(r.nq, r.gates[g], (int64_t)r.mats.size(), &bg[g]);
      if (rc) return rc;
      bg[g].mat_off += mat_base;
    }
    std::vector<double2> m2(r.mats.size());
    for (size_t i = 0; i < m2.size(); ++i) m2[i] = make_double2(r.mats[i].re, r.mats[i].im);
    char *base = (char *)arena_;
    if (hipMemcpyAsync(base + off, r.psi0.data(), (size_t)16 << r.nq, hipMemcpyHostToDevice,
                       stream_) != hipSuccess ||
        (r.ngates && hipMemcpyAsync(base + off + sbytes, bg.data(), bg.size() * sizeof(BGate),
                                    hipMemcpyHostToDevice, stream_) != hipSuccess) ||
        (!m2.empty() && hipMemcpyAsync(base + off + sbytes + gbytes, m2.data(),
                                       m2.size() * sizeof(double2), hipMemcpyHostToDevice,
                                       stream_) != hipSuccess))
      return hip_fail("request upload");
    // The host vectors die with this call: make sure the copies have consumed them.
    if (hipStreamSynchronize(stream_) != hipSuccess) return hip_fail("upload sync");
    return QCW_OK;
  }

  int tick(const std::vector<TickItem> &items) override {
    (void)hipSetDevice(dev_);
    const int n = (int)items.size();
    int max_nq = 1;
    for (int i = 0; i < n; ++i) {
      const SlotInfo &s = slots_[items[i].slot];
      inst_h_[i] = {s.nq, s.ngates, s.state_off, s.gate_off};
      items_h_[i] = {i, tune_.variant[s.nq], items[i].g_begin, items[i].g_end};
      max_nq = std::max(max_nq, s.nq);
    }
    // As in the batched form: exact-kernel items first, then matrix-core
    // items; the most work first in each.
    std::stable_sort(items_h_, items_h_ + n, [&](const BItem &a, const BItem &b) {
      const bool ma = a.variant == kVarAmp4Mfma, mb = b.variant == kVarAmp4Mfma;
      if (ma != mb) return mb;
      return ((int64_t)(a.g_end - a.g_begin) << inst_h_[a.inst].nq) >
             ((int64_t)(b.g_end - b.g_begin) << inst_h_[b.inst].nq);
    });
    int n_exact = 0;
    for (int i = 0; i < n; ++i) n_exact += items_h_[i].variant != kVarAmp4Mfma;
    BatchLaunch L{};
    int rc = plan(max_nq, n_exact, n - n_exact, &L);
    if (rc) return rc;
    L.items = items_d_;
    L.nitems = n;
    L.n_exact = n_exact;
    L.inst = inst_d_;
    L.gates = (const BGate *)arena_;
    L.mats = (const double2 *)arena_;
    L.states = (double2 *)arena_;
    L.counter = counter_d_;
    if (hipMemcpyAsync(inst_d_, inst_h_, sizeof(BInst) * n, hipMemcpyHostToDevice, stream_) !=
            hipSuccess ||
        hipMemcpyAsync(items_d_, items_h_, sizeof(BItem) * n, hipMemcpyHostToDevice, stream_) !=
            hipSuccess)
      return hip_fail("tick tables");
    if ((rc = launch_batch(L, stream_))) return rc;
    for (const TickItem &it : items) {
      if (!it.finishes) continue;
      const SlotInfo &s = slots_[it.slot];
      if (hipMemcpyAsync(result_h_ + ((size_t)it.slot << max_nq_),
                         (char *)arena_ + (uint64_t)s.state_off * 16, (size_t)16 << s.nq,
                         hipMemcpyDeviceToHost, stream_) != hipSuccess)
        return hip_fail("result copy");
    }
    if (hipEventRecord(done_, stream_) != hipSuccess) return hip_fail("event record");
    if (hipEventSynchronize(done_) != hipSuccess) return hip_fail("tick");
    return QCW_OK;
  }

  int fetch(int slot, int nq, qcw_c64 *out) override {
    memcpy(out, result_h_ + ((size_t)slot << max_nq_), (size_t)16 << nq);
    return QCW_OK;
  }

  void release(int slot) override { slots_[slot] = SlotInfo{}; }

 private:
  struct SlotInfo {
    int nq = 0, ngates = 0;
    int64_t state_off = 0, gate_off = 0;
  };

  int plan(int max_nq, int n_exact, int n_mfma, BatchLaunch *L) {
    auto &c = plans_[max_nq];
    if (!c.valid) {
      // Size both grids once per LDS footprint for the largest possible tick.
      int rc = plan_batch_launch(max_nq, max_slots_, max_slots_, &c.L);
      if (rc) return rc;
      c.valid = true;
    }
    *L = c.L;
    auto clamp = [](BatchShape &sh, int items) {
      const int wpb = sh.threads / 64;
      sh.blocks = items > 0 ? (unsigned)std::max(1, std::min<int>((int)sh.blocks, (items + wpb - 1) / wpb)) : 0u;
    };
    clamp(L->ex, n_exact);
    clamp(L->mf, n_mfma);
    return QCW_OK;
  }

  int hip_fail(const char *what) {
    hipError_t e = hipGetLastError();
    return fail(QCW_EHIP, "server %s: %s", what, hipGetErrorString(e));
  }
  int mem_fail(const char *what, uint64_t bytes) {
    (void)hipGetLastError();
    return fail(QCW_ENOMEM, "server %s allocation failed (%llu B)", what, (unsigned long long)bytes);
  }

  struct PlanCache {
    bool valid = false;
    BatchLaunch L{};
  };
  int dev_ = 0;
  int max_slots_ = 0, max_nq_ = 0;
  TuneTable tune_;
  hipStream_t stream_ = nullptr;
  hipEvent_t done_ = nullptr;
  void *arena_ = nullptr;
  uint64_t arena_bytes_ = 0;
  BInst *inst_d_ = nullptr, *inst_h_ = nullptr;
  BItem *items_d_ = nullptr, *items_h_ = nullptr;
  int *counter_d_ = nullptr;
  qcw_c64 *result_h_ = nullptr;
  std::vector<SlotInfo> slots_;
  PlanCache plans_[kBatchMaxNq + 1];
};

}  // namespace
}  // namespace qcw

using namespace qcw;

struct qcw_server {
  std::unique_ptr<ServerCore> core;
};

extern "C" {

int qcw_server_create(qcw_server **out, const qcw_server_cfg *cfg) {
  clear_error();
  if (!out || !cfg) return fail(QCW_EINVAL, "NULL argument");
  *out = nullptr;
  if (cfg->max_slots < 1 || cfg->max_slots > 65536)
    return fail(QCW_EINVAL, "max_slots=%d outside [1, 65536]", cfg->max_slots);
  if (cfg->max_nq < 1 || cfg->max_nq > 11)
    return fail(QCW_EINVAL, "max_nq=%d outside [1, 11]", cfg->max_nq);
  if (cfg->gates_per_tick < 0) return fail(QCW_EINVAL, "gates_per_tick < 0");
  if (cfg->hbm_budget_bytes < 256) return fail(QCW_EINVAL, "hbm_budget_bytes too small");
  ServerConfig sc;
  sc.hbm_budget_bytes = cfg->hbm_budget_bytes;
  sc.max_slots = cfg->max_slots;
  sc.gates_per_tick = cfg->gates_per_tick;
  sc.max_nq = cfg->max_nq;
  auto ex = std::make_unique<HipExecutor>();
  int rc = ex->init(sc, cfg->tune_table);
  if (rc) return rc;
  qcw_server *s = new qcw_server();
  s->core = std::make_unique<ServerCore>(sc, std::move(ex));
  *out = s;
  return QCW_OK;
}

int qcw_server_submit(qcw_server *s, const qcw_request *r, uint64_t *ticket) {
  clear_error();
  if (!s || !r) return fail(QCW_EINVAL, "NULL argument");
  return s->core->submit(*r, ticket);
}

int qcw_server_poll(qcw_server *s, uint64_t ticket, qcw_c64 *psi_out_host, qcw_req_stats *st) {
  clear_error();
  if (!s) return fail(QCW_EINVAL, "NULL server");
  return s->core->poll(ticket, psi_out_host, st);
}

int qcw_server_wait(qcw_server *s, uint64_t ticket, qcw_c64 *psi_out_host, qcw_req_stats *st,
                    double timeout_s) {
  clear_error();
  if (!s) return fail(QCW_EINVAL, "NULL server");
  return s->core->wait(ticket, psi_out_host, st, timeout_s);
}

int qcw_server_counters_get(qcw_server *s, qcw_server_counters *out) {
  clear_error();
  if (!s || !out) return fail(QCW_EINVAL, "NULL argument");
  ServerCounters c = s->core->counters();
  out->submitted = c.submitted;
  out->completed = c.completed;
  out->rejected = c.rejected;
  out->ticks = c.ticks;
  out->peak_active = c.peak_active;
  out->peak_pending = c.peak_pending;
  out->admit_waits = c.admit_waits;
  return QCW_OK;
}

int qcw_server_destroy(qcw_server *s) {
  clear_error();
  if (!s) return QCW_OK;
  s->core->stop();
  delete s;
  return QCW_OK;
}

}  // extern "C"

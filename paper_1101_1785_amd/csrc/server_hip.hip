// GPU executor of the continuous-batching request loop and its C ABI.
//
// Device memory: one arena of the configured budget.  An admitted request
// occupies [state | gate table | matrices] at its arena offset until it
// completes, so its state stays resident across ticks.
//
// Host traffic is batched per tick.  Admission packs each request's region,
// laid out as in the arena, into a pinned staging buffer and returns without
// touching the GPU.  A tick then appends its small tables (copy lists, work
// items) behind the staged requests and issues, on one stream: one
// host-to-device copy of the staging buffer into its device mirror, a
// copy-list kernel that scatters the staged requests into their arena
// regions, ONE persistent batch launch (the same kernel as qcw_batch_run) over
// the resident requests, a copy-list kernel that gathers the states of
// finishing requests into one contiguous buffer, one device-to-host copy of
// that buffer into pinned memory, and an event.  The launch returns; the
// scheduler packs the next tick's requests into a second staging buffer while
// this one runs, and waits for the event before the next launch.
#include <hip/hip_runtime.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <memory>
#include <vector>

#include "qcw_batch.h"
#include "server_core.h"

namespace qcw {

namespace {

uint64_t round256(uint64_t x) { return (x + 255) & ~uint64_t(255); }

static_assert(sizeof(qcw_c64) == sizeof(double2), "qcw_c64 is stored as double2");

// One contiguous device-to-device copy of `bytes` (a multiple of 16) bytes.
struct CopyEnt {
  uint64_t src, dst, bytes, pad;
};
static_assert(sizeof(CopyEnt) == 32, "CopyEnt layout");

constexpr int kCopyThreads = 256;
constexpr int kCopyMaxSplit = 64;                  // blocks per entry at most
constexpr uint64_t kStageBlobBytes = 64ull << 20;  // staged requests between two ticks

// Block (x, y) copies the 16-byte words y*256 + t, stepping 256*gridDim.y, of
// entry x.
__global__ void __launch_bounds__(kCopyThreads) copy_list_kernel(const CopyEnt *__restrict__ ents) {
  const CopyEnt e = ents[blockIdx.x];
  const uint4 *__restrict__ src = (const uint4 *)e.src;
  uint4 *__restrict__ dst = (uint4 *)e.dst;
  const uint64_t words = e.bytes >> 4;
  const uint64_t step = (uint64_t)kCopyThreads * gridDim.y;
  for (uint64_t i = (uint64_t)blockIdx.y * kCopyThreads + threadIdx.x; i < words; i += step)
    dst[i] = src[i];
}

class HipExecutor : public Executor {
 public:
  ~HipExecutor() override {
    if (stream_) (void)hipStreamSynchronize(stream_);
    (void)hipFree(arena_);
    (void)hipFree(res_d_);
    (void)hipFree(counter_d_);
    for (int b = 0; b < 2; ++b) {
      (void)hipFree(mirror_buf_[b]);
      (void)hipHostFree(stage_buf_[b]);
    }
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
    // Every state that finishes in one tick was resident in the arena.
    res_cap_ = std::min<uint64_t>(arena_bytes_, (uint64_t)max_slots_ * (16ull << max_nq_));
    blob_cap_ = std::min<uint64_t>(arena_bytes_, kStageBlobBytes);
    const uint64_t ms = (uint64_t)max_slots_;
    table_cap_ = 2 * round256(ms * sizeof(CopyEnt)) + round256(ms * sizeof(BItem));
    if (hipMalloc(&arena_, std::max<uint64_t>(arena_bytes_, 256)) != hipSuccess)
      return mem_fail("arena", arena_bytes_);
    for (int b = 0; b < 2; ++b)
      if (hipMalloc(&mirror_buf_[b], blob_cap_ + table_cap_) != hipSuccess ||
          hipHostMalloc(&stage_buf_[b], blob_cap_ + table_cap_) != hipSuccess)
        return mem_fail("staging buffers", 2 * (blob_cap_ + table_cap_));
    stage_h_ = stage_buf_[0];
    mirror_d_ = mirror_buf_[0];
    if (hipMalloc(&res_d_, std::max<uint64_t>(res_cap_, 256)) != hipSuccess ||
        hipMalloc(&counter_d_, 2 * sizeof(int)) != hipSuccess)
      return mem_fail("result and counters", res_cap_);
    if (hipHostMalloc(&result_h_, std::max<uint64_t>(res_cap_, 256)) != hipSuccess)
      return mem_fail("pinned result buffer", res_cap_);
    slots_.resize(max_slots_);
    ups_.reserve(max_slots_);
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

  // Packs the request into the staging buffer; the next tick uploads it.
  int load(int slot, uint64_t off, const ServeRequest &r) override {
    (void)hipSetDevice(dev_);
    if (sticky_) return sticky_fail();
    const uint64_t sbytes = round256((uint64_t)16 << r.nq);
    const uint64_t gbytes = round256((uint64_t)sizeof(BGate) * r.ngates);
    const uint64_t need = request_device_bytes(r.nq, r.ngates, (int64_t)r.mats.size());
    if ((off & 255) || off > arena_bytes_ || need > arena_bytes_ - off)
      return fail(QCW_EINVAL, "server: arena region [%llu, +%llu) outside the arena",
                  (unsigned long long)off, (unsigned long long)need);
    const int64_t mat_base = (int64_t)((off + sbytes + gbytes) / 16);
    const bool staged = need <= blob_cap_;
    char *h = nullptr;
    std::vector<char> own;
    if (staged) {
      if (need > blob_cap_ - blob_used_ || (int)ups_.size() == max_slots_) {
        int rc = flush_uploads();
        if (rc) return rc;
      }
      h = stage_h_ + blob_used_;
    } else {
      own.resize(need);  // larger than the staging buffer: uploaded on its own
      h = own.data();
    }
    memcpy(h, r.psi0.data(), (size_t)16 << r.nq);
    BGate *bg = (BGate *)(h + sbytes);
    for (int g = 0; g < r.ngates; ++g) {
      int rc = make_bgate(r.nq, r.gates[g], (int64_t)r.mats.size(), &bg[g]);
      if (rc) return rc;
      bg[g].mat_off += mat_base;
    }
    if (!r.mats.empty()) memcpy(h + sbytes + gbytes, r.mats.data(), 16 * r.mats.size());
    SlotInfo &s = slots_[slot];
    s.nq = r.nq;
    s.ngates = r.ngates;
    s.kmat.resize(r.ngates);
    for (int g = 0; g < r.ngates; ++g) s.kmat[g] = {bg[g].k, bg[g].mat_off};
    s.state_off = (int64_t)(off / 16);
    s.gate_off = (int64_t)((off + sbytes) / 64);
    if (!staged) {
      if (hipMemcpyAsync((char *)arena_ + off, h, need, hipMemcpyHostToDevice, stream_) !=
              hipSuccess ||
          hipStreamSynchronize(stream_) != hipSuccess)
        return bail(hip_fail("request upload"));
      return QCW_OK;
    }
    ups_.push_back({blob_used_, off, need});
    blob_used_ += need;
    return QCW_OK;
  }

  int launch(const std::vector<TickItem> &items) override {
    (void)hipSetDevice(dev_);
    if (sticky_) return sticky_fail();
    const int n = (int)items.size();
    if (n < 1 || n > max_slots_) return bail(fail(QCW_EINVAL, "server: tick of %d items", n));
    // Tables behind the staged requests: [uploads | gathers | items].
    const uint64_t t_up = blob_used_;
    const uint64_t t_ga = t_up + round256(ups_.size() * sizeof(CopyEnt));
    const uint64_t t_it = t_ga + round256((uint64_t)n * sizeof(CopyEnt));
    const uint64_t t_end = t_it + round256((uint64_t)n * sizeof(BItem));
    fill_uploads((CopyEnt *)(stage_h_ + t_up));
    BItem *items_h = (BItem *)(stage_h_ + t_it);
    int max_nq = 1;
    for (int i = 0; i < n; ++i) {
      const SlotInfo &s = slots_[items[i].slot];
      const int gb = items[i].g_begin, ge = items[i].g_end;
      const bool g0 = gb < ge, g1 = gb + 1 < ge;
      items_h[i] = {s.nq, tune_.variant[s.nq], gb, ge, s.state_off, s.gate_off,
                    g0 ? s.kmat[gb].second : 0, g1 ? s.kmat[gb + 1].second : 0,
                    g0 ? s.kmat[gb].first : 0, g1 ? s.kmat[gb + 1].first : 0, {0, 0}};
      max_nq = std::max(max_nq, s.nq);
    }
    // As in the batched form: exact-kernel items first, then matrix-core
    // items; the most work first in each.
    std::stable_sort(items_h, items_h + n, [&](const BItem &a, const BItem &b) {
      const bool ma = a.variant == kVarAmp4Mfma, mb = b.variant == kVarAmp4Mfma;
      if (ma != mb) return mb;
      return ((int64_t)(a.g_end - a.g_begin) << a.nq) > ((int64_t)(b.g_end - b.g_begin) << b.nq);
    });
    int n_exact = 0;
    for (int i = 0; i < n; ++i) n_exact += items_h[i].variant != kVarAmp4Mfma;
    // States of finishing requests, packed one after another.
    CopyEnt *ga = (CopyEnt *)(stage_h_ + t_ga);
    int nga = 0;
    uint64_t res_bytes = 0, ga_max = 0;
    for (const TickItem &it : items) {
      if (!it.finishes) continue;
      SlotInfo &s = slots_[it.slot];
      const uint64_t b = (uint64_t)16 << s.nq, src = (uint64_t)s.state_off * 16;
      if (src > arena_bytes_ || b > arena_bytes_ - src || b > res_cap_ - res_bytes)
        return bail(fail(QCW_EINVAL, "server: result copy outside its buffers"));
      ga[nga++] = {(uint64_t)(uintptr_t)arena_ + src, (uint64_t)(uintptr_t)res_d_ + res_bytes, b, 0};
      s.res_off = res_bytes;
      res_bytes += b;
      ga_max = std::max(ga_max, b);
    }
    BatchLaunch L{};
    int rc = plan(max_nq, n_exact, n - n_exact, &L);
    if (rc) return bail(rc);
    char *mir = (char *)mirror_d_;
    L.items = (const BItem *)(mir + t_it);
    L.nitems = n;
    L.n_exact = n_exact;
    L.gates = (const BGate *)arena_;
    L.mats = (const double2 *)arena_;
    L.states = (double2 *)arena_;
    L.counter = counter_d_;
    if (hipMemcpyAsync(mirror_d_, stage_h_, t_end, hipMemcpyHostToDevice, stream_) != hipSuccess)
      return bail(hip_fail("tick upload"));
    if ((rc = launch_copies((const CopyEnt *)(mir + t_up), (int)ups_.size(), up_max_)) ||
        (rc = launch_batch(L, stream_)) ||
        (rc = launch_copies((const CopyEnt *)(mir + t_ga), nga, ga_max)))
      return bail(rc);
    if (res_bytes && hipMemcpyAsync(result_h_, res_d_, res_bytes, hipMemcpyDeviceToHost,
                                    stream_) != hipSuccess)
      return bail(hip_fail("result copy"));
    if (hipEventRecord(done_, stream_) != hipSuccess) return bail(hip_fail("event record"));
    // Requests admitted while this tick runs are packed into the other staging
    // buffer; the tick before this one finished with it (finish() precedes
    // every launch).
    cur_ ^= 1;
    stage_h_ = stage_buf_[cur_];
    mirror_d_ = mirror_buf_[cur_];
    ups_.clear();
    up_max_ = 0;
    blob_used_ = 0;
    return QCW_OK;
  }

  int finish() override {
    (void)hipSetDevice(dev_);
    if (hipEventSynchronize(done_) != hipSuccess) return bail(hip_fail("tick"));
    return sticky_ ? sticky_fail() : QCW_OK;
  }

  int fetch(int slot, int nq, qcw_c64 *out) override {
    memcpy(out, (const char *)result_h_ + slots_[slot].res_off, (size_t)16 << nq);
    return QCW_OK;
  }

  void release(int slot) override { slots_[slot] = SlotInfo{}; }

 private:
  struct SlotInfo {
    int nq = 0, ngates = 0;
    int64_t state_off = 0, gate_off = 0;
    uint64_t res_off = 0;  // of the final state in the result buffer
    std::vector<std::pair<int, int64_t>> kmat;  // each gate's k and arena matrix offset
  };
  struct Upload {
    uint64_t stage_off, arena_off, bytes;
  };

  // Copy entries of the staged requests: staging mirror -> arena.
  void fill_uploads(CopyEnt *out) {
    up_max_ = 0;
    for (size_t i = 0; i < ups_.size(); ++i) {
      const Upload &u = ups_[i];
      out[i] = {(uint64_t)(uintptr_t)mirror_d_ + u.stage_off,
                (uint64_t)(uintptr_t)arena_ + u.arena_off, u.bytes, 0};
      up_max_ = std::max(up_max_, u.bytes);
    }
  }

  int launch_copies(const CopyEnt *ents_d, int n, uint64_t max_bytes) {
    if (n <= 0) return QCW_OK;
    const uint64_t per_block = (uint64_t)kCopyThreads * 16 * 4;
    const unsigned split =
        (unsigned)std::min<uint64_t>(kCopyMaxSplit, std::max<uint64_t>(1, (max_bytes + per_block - 1) / per_block));
    hipLaunchKernelGGL(copy_list_kernel, dim3((unsigned)n, split), dim3(kCopyThreads), 0, stream_,
                       ents_d);
    if (hipGetLastError() != hipSuccess) return hip_fail("copy-list launch");
    return QCW_OK;
  }

  // The staging buffer is full before the tick: upload and scatter what it
  // holds, wait for the copy, and start it over.
  int flush_uploads() {
    if (ups_.empty()) return QCW_OK;
    const uint64_t t_up = blob_used_;
    const uint64_t t_end = t_up + round256(ups_.size() * sizeof(CopyEnt));
    fill_uploads((CopyEnt *)(stage_h_ + t_up));
    int rc = QCW_OK;
    if (hipMemcpyAsync(mirror_d_, stage_h_, t_end, hipMemcpyHostToDevice, stream_) != hipSuccess)
      rc = hip_fail("staged upload");
    else if ((rc = launch_copies((const CopyEnt *)((char *)mirror_d_ + t_up), (int)ups_.size(),
                                 up_max_)) == QCW_OK &&
             hipStreamSynchronize(stream_) != hipSuccess)
      rc = hip_fail("staged upload sync");
    ups_.clear();
    up_max_ = 0;
    blob_used_ = 0;
    return rc ? sticky_set(rc) : QCW_OK;
  }

  // A failed upload or tick leaves requests half-loaded: every later load and
  // tick fails.  The staged uploads are dropped, so none can land in arena
  // regions that the scheduler hands out again.
  int sticky_set(int rc) {
    int ok = QCW_OK;
    sticky_.compare_exchange_strong(ok, rc);
    return rc;
  }
  int bail(int rc) {
    ups_.clear();
    up_max_ = 0;
    blob_used_ = 0;
    return sticky_set(rc);
  }
  int sticky_fail() { return fail(sticky_, "server executor failed earlier; restart the server"); }

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
  // Staging: requests packed since the last launch [0, blob_used_), then the
  // tick's tables; mirror_d_ is its device copy.  Two such buffers in turn, so
  // requests are packed into one while the tick launched from the other runs.
  char *stage_buf_[2] = {nullptr, nullptr};
  void *mirror_buf_[2] = {nullptr, nullptr};
  int cur_ = 0;
  char *stage_h_ = nullptr;  // = stage_buf_[cur_]
  void *mirror_d_ = nullptr; // = mirror_buf_[cur_]
  uint64_t blob_cap_ = 0, table_cap_ = 0, blob_used_ = 0, up_max_ = 0;
  std::vector<Upload> ups_;
  // Final states of the last tick's finishing requests.
  void *res_d_ = nullptr;
  qcw_c64 *result_h_ = nullptr;
  uint64_t res_cap_ = 0;
  int *counter_d_ = nullptr;
  std::atomic<int> sticky_{QCW_OK};  // read by the waiter thread in finish()
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

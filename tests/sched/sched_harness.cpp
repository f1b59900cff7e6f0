// Test double for the serving scheduler: the real ServerCore driven by an
// executor that performs no arithmetic (a request's "result" is its input
// state) but checks the scheduler's use of device memory -- resident requests
// must occupy disjoint arena regions inside the budget -- and can fail the
// upload of one chosen request, as a device error would.  Built with g++ by
// the CPU tests; never part of the library.
#include <stdint.h>
#include <string.h>

#include <chrono>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "qcw_common.h"
#include "server_core.h"

using namespace qcw;

namespace {

struct Shared {
  std::mutex mu;
  uint64_t budget = 0;
  std::map<int, std::pair<uint64_t, uint64_t>> resident;  // slot -> [off, end)
  int violations = 0;
  int max_tick = 0;
  int ticks = 0;
  uint64_t fail_ticket = 0;
  double tick_seconds = 0;
};

class FakeExecutor : public Executor {
 public:
  explicit FakeExecutor(std::shared_ptr<Shared> sh, int max_slots) : sh_(sh), st_(max_slots) {}
  int load(int slot, uint64_t off, const ServeRequest &r) override {
    std::lock_guard<std::mutex> lk(sh_->mu);
    const uint64_t end = off + request_device_bytes(r.nq, r.ngates, (int64_t)r.mats.size());
    if (end > sh_->budget) sh_->violations++;
    for (auto &kv : sh_->resident)
      if (off < kv.second.second && kv.second.first < end) sh_->violations++;
    if (sh_->resident.count(slot)) sh_->violations++;
    if (r.ticket == sh_->fail_ticket) return fail(QCW_EHIP, "injected upload failure");
    sh_->resident[slot] = {off, end};
    st_[slot] = r.psi0;
    return QCW_OK;
  }
  // A tick may only list resident slots, each continuing exactly where its
  // previous tick left it; at most one tick is in flight.
  int launch(const std::vector<TickItem> &items) override {
    std::lock_guard<std::mutex> lk(sh_->mu);
    if (inflight_) sh_->violations++;
    inflight_ = true;
    sh_->ticks++;
    sh_->max_tick = std::max(sh_->max_tick, (int)items.size());
    for (const TickItem &it : items) {
      if (!sh_->resident.count(it.slot) || it.g_begin > it.g_end) sh_->violations++;
      auto p = progress_.find(it.slot);
      if (it.g_begin != (p == progress_.end() ? 0 : p->second)) sh_->violations++;
      progress_[it.slot] = it.g_end;
    }
    return QCW_OK;
  }
  int finish() override {
    if (sh_->tick_seconds > 0)
      std::this_thread::sleep_for(std::chrono::duration<double>(sh_->tick_seconds));
    std::lock_guard<std::mutex> lk(sh_->mu);
    if (!inflight_) sh_->violations++;
    inflight_ = false;
    return QCW_OK;
  }
  int fetch(int slot, int nq, qcw_c64 *out) override {
    memcpy(out, st_[slot].data(), sizeof(qcw_c64) << nq);
    return QCW_OK;
  }
  void release(int slot) override {
    std::lock_guard<std::mutex> lk(sh_->mu);
    sh_->resident.erase(slot);
    progress_.erase(slot);
  }

 private:
  std::shared_ptr<Shared> sh_;
  std::vector<std::vector<qcw_c64>> st_;
  std::map<int, int> progress_;  // slot -> gates covered by launched ticks
  bool inflight_ = false;
};

struct Harness {
  std::shared_ptr<Shared> sh;
  std::unique_ptr<ServerCore> core;
};

}  // namespace

extern "C" {

void *qcws_create(uint64_t budget, int max_slots, int gates_per_tick, int max_nq,
                  double tick_seconds, uint64_t fail_ticket) {
  auto *h = new Harness();
  h->sh = std::make_shared<Shared>();
  h->sh->budget = budget;
  h->sh->tick_seconds = tick_seconds;
  h->sh->fail_ticket = fail_ticket;
  ServerConfig c;
  c.hbm_budget_bytes = budget;
  c.max_slots = max_slots;
  c.gates_per_tick = gates_per_tick;
  c.max_nq = max_nq;
  h->core = std::make_unique<ServerCore>(c, std::make_unique<FakeExecutor>(h->sh, max_slots));
  return h;
}

int qcws_submit(void *h, const qcw_request *r, uint64_t *t) {
  clear_error();
  return static_cast<Harness *>(h)->core->submit(*r, t);
}

int qcws_poll(void *h, uint64_t t, qcw_c64 *out, qcw_req_stats *st) {
  clear_error();
  return static_cast<Harness *>(h)->core->poll(t, out, st);
}

int qcws_wait(void *h, uint64_t t, qcw_c64 *out, qcw_req_stats *st, double timeout) {
  clear_error();
  return static_cast<Harness *>(h)->core->wait(t, out, st, timeout);
}

int qcws_counters(void *h, qcw_server_counters *o) {
  ServerCounters c = static_cast<Harness *>(h)->core->counters();
  o->submitted = c.submitted;
  o->completed = c.completed;
  o->rejected = c.rejected;
  o->ticks = c.ticks;
  o->peak_active = c.peak_active;
  o->peak_pending = c.peak_pending;
  o->admit_waits = c.admit_waits;
  return 0;
}

int qcws_violations(void *h) {
  auto *x = static_cast<Harness *>(h);
  std::lock_guard<std::mutex> lk(x->sh->mu);
  return x->sh->violations;
}

int qcws_max_tick(void *h) {
  auto *x = static_cast<Harness *>(h);
  std::lock_guard<std::mutex> lk(x->sh->mu);
  return x->sh->max_tick;
}

void qcws_stop(void *h) { static_cast<Harness *>(h)->core->stop(); }

void qcws_destroy(void *h) { delete static_cast<Harness *>(h); }

const char *qcws_last_error(void) { return last_error(); }

}  // extern "C"

// Continuous-batching scheduler (host only).  See server_core.h.
#include "server_core.h"

#include <string.h>
#include <time.h>

#include <algorithm>
#include <chrono>

#include "qcw_common.h"

namespace qcw {

static uint64_t round256(uint64_t x) { return (x + 255) & ~uint64_t(255); }

uint64_t request_device_bytes(int nq, int ngates, int64_t nmats) {
  return round256((uint64_t)16 << nq) + round256((uint64_t)64 * (uint64_t)ngates) +
         round256((uint64_t)16 * (uint64_t)std::max<int64_t>(nmats, 0));
}

// ------------------------------------------------------------------ arena
ArenaAllocator::ArenaAllocator(uint64_t size) : free_bytes_(size & ~uint64_t(255)) {
  if (free_bytes_) free_[0] = free_bytes_;
}

bool ArenaAllocator::alloc(uint64_t bytes, uint64_t *off) {
  bytes = round256(bytes);
  for (auto it = free_.begin(); it != free_.end(); ++it) {
    if (it->second >= bytes) {
      *off = it->first;
      uint64_t rest = it->second - bytes;
      uint64_t roff = it->first + bytes;
      free_.erase(it);
      if (rest) free_[roff] = rest;
      free_bytes_ -= bytes;
      return true;
    }
  }
  return false;
}

void ArenaAllocator::free(uint64_t off, uint64_t bytes) {
  bytes = round256(bytes);
  free_bytes_ += bytes;
  auto it = free_.emplace(off, bytes).first;
  auto nx = std::next(it);
  if (nx != free_.end() && it->first + it->second == nx->first) {
    it->second += nx->second;
    free_.erase(nx);
  }
  if (it != free_.begin()) {
    auto pv = std::prev(it);
    if (pv->first + pv->second == it->first) {
      pv->second += it->second;
      free_.erase(it);
    }
  }
}

// ------------------------------------------------------------------ server
uint64_t ServerCore::now_ns() {
  struct timespec ts;
  clock_gettime(CLOCK_MONOTONIC, &ts);
  return (uint64_t)ts.tv_sec * 1000000000ull + (uint64_t)ts.tv_nsec;
}

ServerCore::ServerCore(const ServerConfig &cfg, std::unique_ptr<Executor> ex)
    : cfg_(cfg), ex_(std::move(ex)), arena_(cfg.hbm_budget_bytes) {
  slots_.resize(cfg_.max_slots);
  for (int i = cfg_.max_slots - 1; i >= 0; --i) free_slots_.push_back(i);
  thr_ = std::thread([this] { loop(); });
  waiter_ = std::thread([this] { wait_ticks(); });
}

ServerCore::~ServerCore() { stop(); }

void ServerCore::stop() {
  {
    std::lock_guard<std::mutex> lk(mu_);
    stop_ = true;
  }
  cv_work_.notify_all();
  cv_tick_.notify_all();
  if (thr_.joinable()) thr_.join();
  if (waiter_.joinable()) waiter_.join();
  std::lock_guard<std::mutex> lk(mu_);
  // Requests still queued or resident when the loop stops fail.
  for (auto &kv : reqs_)
    if (kv.second->status == QCW_EAGAIN) kv.second->status = QCW_EINVAL;
  pending_.clear();
  cv_done_.notify_all();
}

static int validate_request(const qcw_request &r, const ServerConfig &cfg) {
  if (r.nq < 1 || r.nq > cfg.max_nq)
    return fail(QCW_EINVAL, "request nq=%d outside [1, %d]", r.nq, cfg.max_nq);
  if (r.ngates < 0 || r.nmats < 0) return fail(QCW_EINVAL, "negative gate or matrix count");
  if (!r.psi0 || (r.ngates > 0 && (!r.gates || !r.mats)))
    return fail(QCW_EINVAL, "NULL request array");
  for (int g = 0; g < r.ngates; ++g) {
    Geom geo;
    int rc = make_geom(r.nq, r.gates[g].k, r.gates[g].q, &geo);
    if (rc) {
      char why[400];
      snprintf(why, sizeof why, "%s", last_error());
      return fail(rc, "gate %d: %s", g, why);
    }
    const int64_t mm = (int64_t)1 << (2 * r.gates[g].k);
    if (r.gates[g].mat < 0 || r.gates[g].mat + mm > r.nmats)
      return fail(QCW_EINVAL, "gate %d: matrix offset outside mats", g);
  }
  const uint64_t need = request_device_bytes(r.nq, r.ngates, r.nmats);
  if (need > (cfg.hbm_budget_bytes & ~uint64_t(255)))
    return fail(QCW_EINVAL, "request needs %llu B, more than the whole budget",
                (unsigned long long)need);
  return QCW_OK;
}

int ServerCore::submit(const qcw_request &r, uint64_t *ticket) {
  if (!ticket) return fail(QCW_EINVAL, "ticket is NULL");
  int rc = validate_request(r, cfg_);
  if (rc) {
    std::lock_guard<std::mutex> lk(mu_);
    ctr_.rejected++;
    return rc;
  }
  auto q = std::make_unique<ServeRequest>();
  q->nq = r.nq;
  q->ngates = r.ngates;
  q->gates.assign(r.gates, r.gates + r.ngates);
  q->mats.assign(r.mats, r.mats + r.nmats);
  q->psi0.assign(r.psi0, r.psi0 + ((size_t)1 << r.nq));
  q->t_submit = now_ns();
  rc = ex_->prepare(q.get());
  if (!rc && request_device_bytes(q->nq, q->ngates, (int64_t)q->mats.size()) >
                 (cfg_.hbm_budget_bytes & ~uint64_t(255)))
    rc = fail(QCW_EINVAL, "request needs more than the whole budget");
  if (rc) {
    std::lock_guard<std::mutex> lk(mu_);
    ctr_.rejected++;
    return rc;
  }
  {
    std::lock_guard<std::mutex> lk(mu_);
    if (stop_) return fail(QCW_EINVAL, "server is stopping");
    q->ticket = next_ticket_++;
    *ticket = q->ticket;
    pending_.push_back(q->ticket);
    reqs_[q->ticket] = std::move(q);
    ctr_.submitted++;
    ctr_.peak_pending = std::max<uint64_t>(ctr_.peak_pending, pending_.size());
  }
  cv_work_.notify_one();
  return QCW_OK;
}

static void fill_stats(const ServeRequest &q, qcw_req_stats *st) {
  if (!st) return;
  st->status = q.status;
  st->ticks = q.ticks;
  st->t_submit_ns = q.t_submit;
  st->t_admit_ns = q.t_admit;
  st->t_done_ns = q.t_done;
}

int ServerCore::poll(uint64_t ticket, qcw_c64 *psi_out, qcw_req_stats *st) {
  std::lock_guard<std::mutex> lk(mu_);
  auto it = reqs_.find(ticket);
  if (it == reqs_.end()) return fail(QCW_EINVAL, "unknown ticket %llu", (unsigned long long)ticket);
  ServeRequest &q = *it->second;
  fill_stats(q, st);
  if (q.status == QCW_EAGAIN) return QCW_EAGAIN;
  const int rc = q.status;
  if (rc == QCW_OK && psi_out) memcpy(psi_out, q.result.data(), q.result.size() * sizeof(qcw_c64));
  if (rc != QCW_OK) fail(rc, "request %llu failed", (unsigned long long)ticket);
  reqs_.erase(it);
  return rc;
}

int ServerCore::wait(uint64_t ticket, qcw_c64 *psi_out, qcw_req_stats *st, double timeout_s) {
  const auto deadline =
      std::chrono::steady_clock::now() + std::chrono::duration<double>(std::max(0.0, timeout_s));
  {
    std::unique_lock<std::mutex> lk(mu_);
    cv_done_.wait_until(lk, deadline, [&] {
      auto it = reqs_.find(ticket);
      return it == reqs_.end() || it->second->status != QCW_EAGAIN;
    });
  }
  return poll(ticket, psi_out, st);
}

ServerCounters ServerCore::counters() {
  std::lock_guard<std::mutex> lk(mu_);
  return ctr_;
}

// Strict arrival order: the head is admitted when a slot and its memory are
// free; nothing behind it may overtake it.
void ServerCore::admit_locked() {
  while (!pending_.empty() && !free_slots_.empty()) {
    ServeRequest &q = *reqs_[pending_.front()];
    const uint64_t need = request_device_bytes(q.nq, q.ngates, (int64_t)q.mats.size());
    uint64_t off = 0;
    if (!arena_.alloc(need, &off)) {
      ctr_.admit_waits++;
      return;
    }
    const int slot = free_slots_.back();
    free_slots_.pop_back();
    Slot &s = slots_[slot];
    s.used = true;
    s.ticket = q.ticket;
    s.off = off;
    s.bytes = need;
    s.progress = 0;
    int rc = ex_->load(slot, off, q);
    pending_.pop_front();
    q.t_admit = now_ns();
    if (rc) {
      q.status = rc;
      q.t_done = q.t_admit;
      arena_.free(off, need);
      s.used = false;
      free_slots_.push_back(slot);
      ex_->release(slot);
      cv_done_.notify_all();
      continue;
    }
    active_++;
    ctr_.peak_active = std::max<uint64_t>(ctr_.peak_active, (uint64_t)active_);
  }
}

namespace {
constexpr uint64_t kAdmitBatch = 32;
constexpr std::chrono::microseconds kAdmitDelay(100);
}  // namespace

// One tick in flight at a time.  While it runs, the scheduler keeps admitting
// arrivals (packing them for upload: the executor's load), so admission work
// overlaps the GPU work; when the waiter thread reports the tick done, the
// scheduler completes its finishing requests (their slots and arena regions
// are freed only now), plans the next tick over every resident request and
// launches it.
void ServerCore::loop() {
  std::vector<TickItem> next, inflight;
  bool running = false;
  for (;;) {
    next.clear();
    {
      std::unique_lock<std::mutex> lk(mu_);
      if (!running) {
        cv_work_.wait(lk, [&] { return stop_ || !pending_.empty() || active_ > 0; });
      } else {
        // While the tick runs, arrivals are admitted in batches: when
        // kAdmitBatch of them have come, or kAdmitDelay after the wait began
        // if any have (one wake-up per arrival would cost more lock traffic
        // than the packing it moves off the critical path).
        cv_work_.wait(lk, [&] {
          return stop_ || tick_done_ || ctr_.submitted != seen_submitted_;
        });
        if (!stop_ && !tick_done_) {
          const auto deadline = std::chrono::steady_clock::now() + kAdmitDelay;
          cv_work_.wait_until(lk, deadline, [&] {
            return stop_ || tick_done_ || ctr_.submitted - seen_submitted_ >= kAdmitBatch;
          });
        }
      }
      if (stop_) {
        // the tick in flight must end before the executor may go away
        cv_work_.wait(lk, [&] { return !running || tick_done_; });
        return;
      }
      if (running && !tick_done_) {
        seen_submitted_ = ctr_.submitted;
        admit_locked();
        continue;
      }
      if (running) {
        complete_locked(inflight, tick_rc_);
        running = false;
        tick_done_ = false;
      }
      seen_submitted_ = ctr_.submitted;
      admit_locked();
      for (int i = 0; i < (int)slots_.size(); ++i) {
        Slot &s = slots_[i];
        if (!s.used) continue;
        ServeRequest &q = *reqs_[s.ticket];
        int end = q.ngates;
        if (cfg_.gates_per_tick > 0) end = std::min(q.ngates, s.progress + cfg_.gates_per_tick);
        next.push_back({i, s.progress, end, end == q.ngates});
        s.progress = end;
      }
    }
    if (next.empty()) continue;
    const int rc = ex_->launch(next);
    std::lock_guard<std::mutex> lk(mu_);
    if (rc) {
      complete_locked(next, rc);
      continue;
    }
    inflight.swap(next);
    running = true;
    tick_launched_ = true;
    cv_tick_.notify_one();
  }
}

// The waiter: blocks in Executor::finish() for each launched tick, then hands
// its status to the scheduler.
void ServerCore::wait_ticks() {
  for (;;) {
    {
      std::unique_lock<std::mutex> lk(mu_);
      cv_tick_.wait(lk, [&] { return tick_launched_ || stop_; });
      if (!tick_launched_) return;  // stopping with no tick in flight
      tick_launched_ = false;
    }
    const int rc = ex_->finish();
    std::lock_guard<std::mutex> lk(mu_);
    tick_rc_ = rc;
    tick_done_ = true;
    cv_work_.notify_all();
  }
}

// Bookkeeping after a tick (rc: its status): finishing requests get their
// results (or the error) and release their slots; with an error every request
// of the tick fails.
void ServerCore::complete_locked(const std::vector<TickItem> &items, int rc) {
  ctr_.ticks++;
  const uint64_t t = now_ns();
  for (const TickItem &it : items) {
    Slot &s = slots_[it.slot];
    if (!s.used) continue;
    ServeRequest &q = *reqs_[s.ticket];
    q.ticks++;
    if (rc == QCW_OK && !it.finishes) continue;
    if (rc == QCW_OK) {
      q.result.resize((size_t)1 << q.nq);
      q.status = ex_->fetch(it.slot, q.nq, q.result.data());
    } else {
      q.status = rc;
    }
    q.t_done = t;
    ctr_.completed++;
    arena_.free(s.off, s.bytes);
    s = Slot{};
    free_slots_.push_back(it.slot);
    ex_->release(it.slot);
    active_--;
  }
  cv_done_.notify_all();
}

}  // namespace qcw

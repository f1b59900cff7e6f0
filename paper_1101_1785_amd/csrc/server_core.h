// Continuous-batching request loop (host only, no HIP): admission of requests
// into device slots under an HBM budget, per-tick planning of which slots
// advance by how many gates, and completion bookkeeping.  The device work is
// behind the Executor interface, so the scheduling logic is the same whether
// the executor drives the GPU or is a test double.
#pragma once

#include <stdint.h>

#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "qcw.h"

namespace qcw {

struct ServeRequest {
  int nq = 0;
  int ngates = 0;
  std::vector<qcw_gate> gates;  // matrix offsets relative to `mats`
  std::vector<qcw_c64> mats;
  std::vector<qcw_c64> psi0;
  uint64_t ticket = 0;
  uint64_t t_submit = 0, t_admit = 0, t_done = 0;
  int status = QCW_EAGAIN;
  int ticks = 0;
  std::vector<qcw_c64> result;
};

// Device bytes a request occupies while resident: state, gate table, matrices
// (each region rounded to 256 bytes).
uint64_t request_device_bytes(int nq, int ngates, int64_t nmats);

struct TickItem {
  int slot;
  int g_begin, g_end;
  bool finishes;
};

class Executor {
 public:
  virtual ~Executor() {}
  // May rewrite a submitted request's circuit into an equivalent one before it
  // is sized and queued (called from the submitting thread).
  virtual int prepare(ServeRequest *r) {
    (void)r;
    return QCW_OK;
  }
  // Copies an admitted request into the arena at `off` (its own region).  It
  // may be called while a launched tick runs: the copy must then not disturb
  // that tick, and it reaches the arena no later than the next launch.
  virtual int load(int slot, uint64_t off, const ServeRequest &r) = 0;
  // Starts one tick: every listed slot advances over its gate range and the
  // states of finishing slots are copied out.  Returns without waiting; at
  // most one tick is in flight, and finish() is called before the next launch.
  virtual int launch(const std::vector<TickItem> &items) = 0;
  // Waits for the launched tick; its results can then be fetched.
  virtual int finish() = 0;
  // The final state of a slot that finished in the last finished tick.
  virtual int fetch(int slot, int nq, qcw_c64 *out) = 0;
  // Releases a slot (its arena region is free again).
  virtual void release(int slot) = 0;
};

// First-fit allocator over [0, size) with coalescing; 256-byte granules.
class ArenaAllocator {
 public:
  explicit ArenaAllocator(uint64_t size);
  bool alloc(uint64_t bytes, uint64_t *off);
  void free(uint64_t off, uint64_t bytes);
  uint64_t free_bytes() const { return free_bytes_; }

 private:
  std::map<uint64_t, uint64_t> free_;  // offset -> length
  uint64_t free_bytes_;
};

struct ServerConfig {
  uint64_t hbm_budget_bytes = 1ull << 30;
  int max_slots = 1024;
  int gates_per_tick = 0;  // 0: a slot runs its remaining gates in one tick
  int max_nq = 11;
};

struct ServerCounters {
  uint64_t submitted = 0, completed = 0, rejected = 0, ticks = 0;
  uint64_t peak_active = 0, peak_pending = 0;
  uint64_t admit_waits = 0;  // ticks in which the queue head could not be admitted
};

class ServerCore {
 public:
  ServerCore(const ServerConfig &cfg, std::unique_ptr<Executor> ex);
  ~ServerCore();
  int submit(const qcw_request &r, uint64_t *ticket);
  // QCW_OK: done (result copied, ticket released); QCW_EAGAIN: pending;
  // another code: the request failed (ticket released).
  int poll(uint64_t ticket, qcw_c64 *psi_out, qcw_req_stats *st);
  int wait(uint64_t ticket, qcw_c64 *psi_out, qcw_req_stats *st, double timeout_s);
  ServerCounters counters();
  void stop();
  static uint64_t now_ns();

 private:
  void loop();
  void wait_ticks();
  void admit_locked();
  void complete_locked(const std::vector<TickItem> &items, int rc);
  struct Slot {
    bool used = false;
    uint64_t ticket = 0;
    uint64_t off = 0, bytes = 0;
    int progress = 0;  // gates covered by the ticks launched so far
  };
  ServerConfig cfg_;
  std::unique_ptr<Executor> ex_;
  std::mutex mu_;
  std::condition_variable cv_work_, cv_done_;
  std::deque<uint64_t> pending_;
  std::unordered_map<uint64_t, std::unique_ptr<ServeRequest>> reqs_;
  std::vector<Slot> slots_;
  std::vector<int> free_slots_;
  ArenaAllocator arena_;
  uint64_t next_ticket_ = 1;
  bool stop_ = false;
  int active_ = 0;
  ServerCounters ctr_;
  // The tick in flight: the scheduler launches it and goes on admitting
  // arrivals; the waiter thread blocks in Executor::finish() and reports.
  bool tick_launched_ = false, tick_done_ = false;
  int tick_rc_ = QCW_OK;
  uint64_t seen_submitted_ = 0;  // submissions the scheduler has looked at
  std::condition_variable cv_tick_;
  std::thread thr_, waiter_;
};

}  // namespace qcw

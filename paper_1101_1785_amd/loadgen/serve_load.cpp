// Open-loop load generator for the request server (qcw_server_*, include/qcw.h).
//
// Submits requests from native client threads at scheduled arrival times, so
// that the server, not a scripting-language client, sets the sustainable
// rate; a collector thread waits for every request in submission order and
// copies its result to host memory, as a caller would.
//
// usage: serve_load POOL ARRIVALS OUT BUDGET_BYTES MAX_SLOTS MAX_NQ TUNE_TABLE|- CLIENTS
//   POOL      requests: int32 count, then per request int32 nq, int32 ngates,
//             int64 nmats, ngates qcw_gate rows (matrix offsets into this
//             request's mats), nmats qcw_c64, 2^nq qcw_c64 (the input state)
//   ARRIVALS  int64 n, then n doubles: arrival times in seconds from the start
//             (request i is pool entry i mod count)
//   OUT       written: int64 n, int64 ticks, int64 peak_active, then per
//             request int64 scheduled_ns, int64 done_ns, int32 status
// Exit status 0 when every request completed.
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>

#include <atomic>
#include <thread>
#include <vector>

#include "qcw.h"

namespace {

struct Request {
  int nq = 0;
  std::vector<qcw_gate> gates;
  std::vector<qcw_c64> mats;
  std::vector<qcw_c64> psi0;
};

uint64_t now_ns() {
  timespec ts;
  clock_gettime(CLOCK_MONOTONIC, &ts);
  return (uint64_t)ts.tv_sec * 1000000000ull + (uint64_t)ts.tv_nsec;
}

void sleep_until(uint64_t t) {
  for (;;) {
    const uint64_t n = now_ns();
    if (n >= t) return;
    const uint64_t d = t - n;
    if (d > 200000) {  // coarse sleep, then spin the last 0.2 ms
      timespec ts{(time_t)((d - 100000) / 1000000000ull), (long)((d - 100000) % 1000000000ull)};
      nanosleep(&ts, nullptr);
    }
  }
}

bool read_exact(FILE *f, void *p, size_t n) { return fread(p, 1, n, f) == n; }

bool read_pool(const char *path, std::vector<Request> *pool) {
  FILE *f = fopen(path, "rb");
  if (!f) return false;
  int32_t count = 0;
  bool ok = read_exact(f, &count, sizeof count) && count > 0;
  for (int32_t i = 0; ok && i < count; ++i) {
    int32_t nq = 0, ng = 0;
    int64_t nm = 0;
    ok = read_exact(f, &nq, 4) && read_exact(f, &ng, 4) && read_exact(f, &nm, 8) && nq >= 1 &&
         nq <= 20 && ng >= 0 && nm >= 0;
    if (!ok) break;
    Request r;
    r.nq = nq;
    r.gates.resize((size_t)ng);
    r.mats.resize((size_t)nm);
    r.psi0.resize((size_t)1 << nq);
    ok = read_exact(f, r.gates.data(), sizeof(qcw_gate) * (size_t)ng) &&
         read_exact(f, r.mats.data(), sizeof(qcw_c64) * (size_t)nm) &&
         read_exact(f, r.psi0.data(), sizeof(qcw_c64) * r.psi0.size());
    pool->push_back(std::move(r));
  }
  fclose(f);
  return ok;
}

bool read_arrivals(const char *path, std::vector<double> *t) {
  FILE *f = fopen(path, "rb");
  if (!f) return false;
  int64_t n = 0;
  bool ok = read_exact(f, &n, 8) && n > 0;
  if (ok) {
    t->resize((size_t)n);
    ok = read_exact(f, t->data(), sizeof(double) * (size_t)n);
  }
  fclose(f);
  return ok;
}

int submit(qcw_server *s, const Request &r, uint64_t *ticket) {
  qcw_request q;
  q.nq = r.nq;
  q.ngates = (int)r.gates.size();
  q.gates = r.gates.empty() ? nullptr : r.gates.data();
  q.mats = r.mats.data();
  q.nmats = (int64_t)r.mats.size();
  q.psi0 = r.psi0.data();
  return qcw_server_submit(s, &q, ticket);
}

}  // namespace

int main(int argc, char **argv) {
  if (argc != 9) {
    fprintf(stderr,
            "usage: %s POOL ARRIVALS OUT BUDGET_BYTES MAX_SLOTS MAX_NQ TUNE_TABLE|- CLIENTS\n",
            argv[0]);
    return 2;
  }
  std::vector<Request> pool;
  std::vector<double> arr;
  if (!read_pool(argv[1], &pool) || !read_arrivals(argv[2], &arr)) {
    fprintf(stderr, "serve_load: cannot read the request pool or the arrivals\n");
    return 2;
  }
  qcw_server_cfg cfg;
  memset(&cfg, 0, sizeof cfg);
  cfg.hbm_budget_bytes = strtoull(argv[4], nullptr, 10);
  cfg.max_slots = atoi(argv[5]);
  cfg.gates_per_tick = 0;
  cfg.max_nq = atoi(argv[6]);
  cfg.tune_table = strcmp(argv[7], "-") ? argv[7] : nullptr;
  const int clients = atoi(argv[8]) > 0 ? atoi(argv[8]) : 1;
  qcw_server *s = nullptr;
  if (qcw_server_create(&s, &cfg) != QCW_OK) {
    fprintf(stderr, "serve_load: server: %s\n", qcw_last_error());
    return 1;
  }
  int max_nq = 1;
  for (const Request &r : pool) max_nq = r.nq > max_nq ? r.nq : max_nq;
  std::vector<qcw_c64> out((size_t)1 << max_nq);
  // warm the path (kernel load, graph capture)
  for (size_t i = 0; i < pool.size() && i < 64; ++i) {
    uint64_t t = 0;
    if (submit(s, pool[i], &t) != QCW_OK ||
        qcw_server_wait(s, t, out.data(), nullptr, 60.0) != QCW_OK) {
      fprintf(stderr, "serve_load: warm-up request failed: %s\n", qcw_last_error());
      qcw_server_destroy(s);
      return 1;
    }
  }
  const size_t n = arr.size();
  const uint64_t t0 = now_ns() + 20000000ull;
  std::vector<uint64_t> sched(n), done(n, 0), tickets(n, 0);
  std::vector<int32_t> status(n, QCW_EAGAIN);
  std::vector<std::atomic<int>> ready(n);
  for (auto &x : ready) x.store(0);
  for (size_t i = 0; i < n; ++i) sched[i] = t0 + (uint64_t)(arr[i] * 1e9);
  std::vector<std::thread> cl;
  for (int c = 0; c < clients; ++c) {
    cl.emplace_back([&, c]() {
      for (size_t i = (size_t)c; i < n; i += (size_t)clients) {
        sleep_until(sched[i]);
        uint64_t t = 0;
        const int rc = submit(s, pool[i % pool.size()], &t);
        tickets[i] = t;
        status[i] = rc == QCW_OK ? QCW_EAGAIN : rc;
        ready[i].store(rc == QCW_OK ? 1 : 2, std::memory_order_release);
      }
    });
  }
  std::thread col([&]() {
    for (size_t i = 0; i < n; ++i) {
      int r;
      while ((r = ready[i].load(std::memory_order_acquire)) == 0) std::this_thread::yield();
      if (r != 1) continue;
      qcw_req_stats st;
      const int rc = qcw_server_wait(s, tickets[i], out.data(), &st, 120.0);
      status[i] = rc;
      done[i] = rc == QCW_OK ? st.t_done_ns : 0;
    }
  });
  for (auto &t : cl) t.join();
  col.join();
  qcw_server_counters cnt;
  memset(&cnt, 0, sizeof cnt);
  qcw_server_counters_get(s, &cnt);
  qcw_server_destroy(s);
  FILE *f = fopen(argv[3], "wb");
  if (!f) return 2;
  const int64_t hdr[3] = {(int64_t)n, (int64_t)cnt.ticks, (int64_t)cnt.peak_active};
  fwrite(hdr, sizeof hdr, 1, f);
  int failed = 0;
  for (size_t i = 0; i < n; ++i) {
    const int64_t a = (int64_t)sched[i], b = (int64_t)done[i];
    fwrite(&a, 8, 1, f);
    fwrite(&b, 8, 1, f);
    fwrite(&status[i], 4, 1, f);
    failed += status[i] != QCW_OK;
  }
  fclose(f);
  return failed ? 1 : 0;
}

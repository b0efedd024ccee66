// Host-thread model of the ready-queue executor protocol (csrc/queue.h),
// built with ThreadSanitizer by tests/test_queue_model.py.
//
// Reads a graph (one task per line: class lane paired items npreds preds...),
// lays it out with the runtime's layout code and runs it with worker threads
// per class executing the same pop / complete protocol as the device
// kernels.  Each item's body writes its own mark with a plain store and
// reads the marks of all items of the task's predecessors with plain loads:
// a missing happens-before edge in the protocol is a data race that
// ThreadSanitizer reports, and a predecessor item found unmarked fails the
// run.  Marks also catch an item run twice.  Exit status 0 and a line
// "ok ..." on success.
//
//   queue_model GRAPH WORKERS_PER_CLASS [stuck_task] [stagger_us] [cus]
// stuck_task >= 0 adds one to that task's dependency count (it can never
// become ready): the run must end through the watchdog, every worker having
// left, with status[0] set.  cus > 0 models the device's CUs: a worker must
// hold one of cus tokens to run, and the classes are started GEMM classes
// first, panel last, so that with fewer tokens than workers the panel
// workers can only run once idle GEMM workers yield their CU.
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include <atomic>
#include <chrono>
#include <condition_variable>
#include <mutex>
#include <fstream>
#include <thread>
#include <vector>

#include "queue_layout.h"

struct HostAT {
  // Every operation is made acquire/release (fences are no-ops): the thread
  // sanitizer does not model fences, and the strengthened operations carry
  // the ordering the device's fences provide.
  template <class T> static T ld(T *p) { return __atomic_load_n(p, __ATOMIC_ACQUIRE); }
  template <class T> static void st(T *p, T v) { __atomic_store_n(p, v, __ATOMIC_RELEASE); }
  template <class T> static bool cas(T *p, T *e, T d) {
    return __atomic_compare_exchange_n(p, e, d, false, __ATOMIC_ACQ_REL, __ATOMIC_ACQUIRE);
  }
  template <class T> static T add(T *p, T v) { return __atomic_fetch_add(p, v, __ATOMIC_ACQ_REL); }
  static void fence_rel() {}
  static void fence_acq() {}
  static uint64_t now() {
    return (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
  }
  static void pause() { std::this_thread::yield(); }
};

int main(int argc, char **argv) {
  if (argc < 3) {
    fprintf(stderr, "usage: queue_model GRAPH WORKERS [stuck_task] [stagger_us]\n");
    return 2;
  }
  std::ifstream in(argv[1]);
  const int workers = atoi(argv[2]);
  const long stuck = argc > 3 ? atol(argv[3]) : -1;
  const long stagger_us = argc > 4 ? atol(argv[4]) : 0;
  const long cus = argc > 5 ? atol(argv[5]) : 0;
  int64_t nt = 0;
  in >> nt;
  std::vector<dcq::TaskIn> tasks(nt);
  std::vector<std::vector<int64_t>> preds(nt);
  for (int64_t t = 0; t < nt; ++t) {
    int64_t np = 0;
    dcq::TaskIn &k = tasks[t];
    in >> k.cls >> k.lane >> k.paired >> k.items >> np;
    preds[t].resize(np);
    for (int64_t i = 0; i < np; ++i) in >> preds[t][i];
    k.preds = preds[t].data();
    k.npreds = np;
  }
  if (!in) { fprintf(stderr, "bad graph file\n"); return 2; }
  dcq::Sizes s;
  if (dcq::layout_sizes(nt, tasks.data(), s)) { fprintf(stderr, "layout_sizes failed\n"); return 2; }
  dcq::Ctl ctl;
  std::vector<int32_t> deps(nt), left(nt), soff(nt + 1), succ(s.nedges + 1);
  std::vector<uint32_t> meta(nt);
  std::vector<uint64_t> ring(s.nitems + 1);
  int32_t status[4] = {0, 0, 0, 0};
  const int64_t watchdog_ns = stuck >= 0 ? 200000000 : 20000000000LL;
  int64_t launched[dcq::NCLASS] = {0, 0, 0, 0};
  for (int64_t t = 0; t < nt; ++t) launched[tasks[t].cls] = workers;
  dcq::layout_fill(nt, tasks.data(), s, watchdog_ns, 20000000, launched,
                   {&ctl, deps.data(), left.data(), soff.data(), succ.data(), meta.data(),
                    ring.data()});
  if (stuck >= 0 && stuck < nt) deps[stuck] += 1;
  dcq::View q{&ctl, deps.data(), left.data(), soff.data(), succ.data(), meta.data(),
              ring.data(), status};

  // plain (non-atomic) marks, one per item
  std::vector<std::vector<uint8_t>> mark(nt);
  for (int64_t t = 0; t < nt; ++t) mark[t].assign(tasks[t].items, 0);
  std::atomic<int64_t> errors{0}, ran{0};

  // CU tokens
  std::mutex mu;
  std::condition_variable cv;
  long tokens = cus;
  std::atomic<int64_t> yielded_or_done{0};
  auto worker = [&](int cls, int id) {
    if (stagger_us > 0)
      std::this_thread::sleep_for(std::chrono::microseconds(stagger_us * (id % 7)));
    if (cus > 0) {
      std::unique_lock<std::mutex> lk(mu);
      cv.wait(lk, [&] { return tokens > 0; });
      --tokens;
    }
    dcq::worker_start<HostAT>(q, cls);
    for (;;) {
      uint64_t it = 0;
      const int r = dcq::pop<HostAT>(q, cls, &it);
      if (r != dcq::POP_ITEM) break;
      const int64_t t = dcq::item_task(it);
      const int u = dcq::item_unit(it);
      const int step = dcq::meta_step(meta[t]);
      if (t < 0 || t >= nt || u % step || u / step >= tasks[t].items ||
          dcq::meta_class(meta[t]) != cls) {
        errors++;
        break;
      }
      for (int64_t i = 0; i < tasks[t].npreds; ++i) {
        const int64_t p = tasks[t].preds[i];
        for (uint8_t m : mark[p])
          if (m != 1) errors++;
      }
      if (mark[t][u / step] != 0) errors++;
      mark[t][u / step] = 1;
      ran++;
      dcq::complete<HostAT>(q, t);
    }
    if (cus > 0) {
      std::lock_guard<std::mutex> lk(mu);
      ++tokens;
      cv.notify_all();
    }
    yielded_or_done++;
  };
  std::vector<std::thread> th;
  for (int cls = dcq::NCLASS - 1; cls >= 0; --cls) {
    if (ctl.total[cls] == 0) continue;
    for (int w = 0; w < workers; ++w) th.emplace_back(worker, cls, w);
    // with modelled CUs, let this class take its tokens before the next one
    if (cus > 0) std::this_thread::sleep_for(std::chrono::milliseconds(20));
  }
  for (auto &x : th) x.join();

  int64_t unmarked = 0;
  for (int64_t t = 0; t < nt; ++t)
    for (uint8_t m : mark[t]) unmarked += m == 0;
  if (stuck >= 0) {
    // the stuck task and everything after it on a path stays undone, the
    // watchdog must have fired and every worker must have left
    if (status[0] != 1 || unmarked == 0 || errors) {
      fprintf(stderr, "watchdog case failed: status %d unmarked %lld errors %lld\n", status[0],
              (long long)unmarked, (long long)errors.load());
      return 1;
    }
    printf("ok watchdog tasks=%lld items_run=%lld unmarked=%lld\n", (long long)nt,
           (long long)ran.load(), (long long)unmarked);
    return 0;
  }
  int64_t heads = 0;
  for (int c = 0; c < dcq::NCLASS; ++c)
    for (int l = 0; l < dcq::NLANE; ++l) heads += (int64_t)ctl.head[c][l].v;
  if (errors || unmarked || status[0] || heads != s.nitems ||
      (int64_t)ctl.completed.v != nt) {
    fprintf(stderr, "failed: errors %lld unmarked %lld status %d heads %lld/%lld completed %lld/%lld\n",
            (long long)errors.load(), (long long)unmarked, status[0], (long long)heads,
            (long long)s.nitems, (long long)ctl.completed.v, (long long)nt);
    return 1;
  }
  printf("ok tasks=%lld edges=%lld items=%lld threads=%zu yielded=%lld\n", (long long)nt,
         (long long)s.nedges, (long long)s.nitems, th.size(), (long long)ctl.yielded.v);
  return 0;
}

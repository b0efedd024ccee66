// Host-side layout of a graph for the ready-queue executor (queue.h): the
// per-task dependency and item counters, the successor lists (CSR), the
// metadata words, the rings with the initially ready tasks' items already in
// place, and the control block.  Plain C++; used by the runtime and by the
// host-thread model of the executor in the tests.
#pragma once
#include <stdint.h>
#include <string.h>

#include <vector>

#include "queue.h"

namespace dcq {

struct TaskIn {
  const int64_t *preds;   // distinct earlier tasks this one depends on
  int64_t npreds;
  int cls;                // worker class (CL_*)
  int lane;               // priority lane, 0 first
  int paired;             // items are pairs of units
  int64_t items;          // work items (>= 1)
};

struct Sizes {
  int64_t ntasks = 0, nedges = 0, nitems = 0;
};

// Counts edges and items; returns 0, or -1 when a count does not fit the
// 32-bit fields of the layout or a task is malformed.
inline int layout_sizes(int64_t nt, const TaskIn *tasks, Sizes &s) {
  s.ntasks = nt;
  s.nedges = 0;
  s.nitems = 0;
  for (int64_t t = 0; t < nt; ++t) {
    const TaskIn &k = tasks[t];
    if (k.items < 1 || k.items >= MAX_ITEMS_PER_TASK || k.cls < 0 || k.cls >= NCLASS ||
        k.lane < 0 || k.lane >= NLANE)
      return -1;
    for (int64_t i = 0; i < k.npreds; ++i)
      if (k.preds[i] < 0 || k.preds[i] >= t) return -1;
    s.nedges += k.npreds;
    s.nitems += k.items;
  }
  if (nt >= INT32_MAX || s.nedges >= INT32_MAX) return -1;
  return 0;
}

// Output arrays (caller-allocated, sizes from layout_sizes).
struct Out {
  Ctl *ctl;
  int32_t *deps, *left, *soff, *succ;   // ntasks, ntasks, ntasks + 1, nedges
  uint32_t *meta;                       // ntasks
  uint64_t *ring;                       // nitems
};

// Fills the layout.  Tasks without predecessors are placed in their lanes'
// rings in submission order (their tails count them).  workers: the
// workers launched per class; yield_ticks: idle time after which a worker
// may give up its CU to a class whose workers have not started.
inline void layout_fill(int64_t nt, const TaskIn *tasks, const Sizes &s, int64_t watchdog_ticks,
                        int64_t yield_ticks, const int64_t *workers, const Out &o) {
  memset((void *)o.ctl, 0, sizeof(Ctl));
  Ctl &c = *o.ctl;
  c.watchdog_ticks = watchdog_ticks;
  c.yield_ticks = yield_ticks;
  for (int k = 0; k < NCLASS; ++k) c.workers[k] = workers[k];
  for (int64_t t = 0; t < nt; ++t) {
    const TaskIn &k = tasks[t];
    c.cap[k.cls][k.lane] += k.items;
    c.total[k.cls] += k.items;
  }
  int64_t b = 0;
  for (int cl = 0; cl < NCLASS; ++cl)
    for (int l = 0; l < NLANE; ++l) {
      c.base[cl][l] = b;
      b += c.cap[cl][l];
    }
  // successor counts, then offsets, then lists (successors in ascending
  // task order, since tasks are visited in submission order)
  std::vector<int32_t> fill(nt + 1, 0);
  for (int64_t t = 0; t < nt; ++t)
    for (int64_t i = 0; i < tasks[t].npreds; ++i) fill[tasks[t].preds[i] + 1] += 1;
  o.soff[0] = 0;
  for (int64_t t = 0; t < nt; ++t) o.soff[t + 1] = o.soff[t] + fill[t + 1];
  for (int64_t t = 0; t < nt; ++t) fill[t] = o.soff[t];
  for (int64_t t = 0; t < nt; ++t) {
    const TaskIn &k = tasks[t];
    for (int64_t i = 0; i < k.npreds; ++i) o.succ[fill[k.preds[i]]++] = (int32_t)t;
    o.deps[t] = (int32_t)k.npreds;
    o.left[t] = (int32_t)k.items;
    o.meta[t] = meta_pack(k.cls, k.lane, k.paired, k.items);
  }
  memset(o.ring, 0, (size_t)s.nitems * sizeof(uint64_t));
  for (int64_t t = 0; t < nt; ++t) {
    const TaskIn &k = tasks[t];
    if (k.npreds) continue;
    uint64_t &tail = c.tail[k.cls][k.lane].v;
    uint64_t *r = o.ring + c.base[k.cls][k.lane] + (int64_t)tail;
    const int step = k.paired ? 2 : 1;
    for (int64_t i = 0; i < k.items; ++i) r[i] = item_enc(t, i * step);
    tail += (uint64_t)k.items;
  }
}

}  // namespace dcq

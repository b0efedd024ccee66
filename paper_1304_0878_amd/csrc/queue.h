// Ready-queue executor: the graph layout it reads and the protocol its
// workers follow (pop a ready work item, run it, complete it, release the
// successors whose dependency count reaches zero).  The dependency counts are
// the access-mode graph of the paper's Section 2 (a task runs once every
// task it depends on has completed); the priority lanes are the scheduling
// hints of its Section 5.3.
//
// The protocol is written once, over an atomics policy AT, so that the same
// code runs in the device kernels (HIP atomics at agent scope) and in a
// host-thread model of the executor used by the tests.  AT provides:
//   ld(p)            relaxed atomic load
//   st(p, v)         relaxed atomic store
//   cas(p, &e, d)    relaxed compare-and-swap (e receives the observed value)
//   add(p, v)        relaxed fetch-and-add, returns the old value
//   fence_rel()      release fence, fence_acq() acquire fence
//   now()            a monotonic tick count, pause() a short back-off
// Ordering follows the fence rules of the C++ memory model: a release fence
// sequenced before an atomic write W synchronizes with an acquire fence
// sequenced after an atomic read that reads W (or a later value of an RMW
// chain on the same object).
//
// Residency: the launches of one graph are sized to fit on the device
// together, but other work on the device (another runtime's graph) can hold
// CUs that a class's workers need, while the other classes' workers wait for
// that class's tasks.  A worker that has been idle for yield_ticks while
// workers of another class of the graph have not started leaves early (at
// most as many as are missing, never the last worker of its class), which
// frees its CU for them.
//
// Termination: every task is pushed exactly once, so each (class, lane) ring
// receives exactly cap items over the graph.  A worker only claims a slot
// that a pusher has already reserved (head < tail), so it never waits for
// work that may not come; it leaves when every item of its class has been
// claimed (sum of heads == class total), which needs no other worker.  Every
// wait is bounded: without progress (no task completed) for watchdog_ticks
// a worker sets the abort word and leaves, and every other worker leaves as
// soon as it sees the word.
#pragma once
#include <stdint.h>

#if defined(__HIPCC__)
#define DCQ_HD __host__ __device__
#else
#define DCQ_HD
#endif

namespace dcq {

constexpr int NCLASS = 4;   // worker kernels: panel, FP64 GEMM, FP32-input GEMM, BF16 GEMM
constexpr int NLANE = 4;    // priority lanes per class; lane 0 is taken first
constexpr int CL_PANEL = 0, CL_G64 = 1, CL_G32 = 2, CL_LOWP = 3;

// One counter per 128-byte line (an L2 line): the claim and reservation
// counters of different lanes are contended independently.
struct alignas(128) Line {
  uint64_t v;
  uint64_t pad[15];
};

// Control block of one graph, written by the host before the launch.
struct Ctl {
  Line head[NCLASS][NLANE];     // ring slots claimed so far
  Line tail[NCLASS][NLANE];     // ring slots reserved by pushers so far
  Line completed;               // tasks completed (progress, for the watchdog)
  Line abort;                   // nonzero: every worker leaves
  Line started[NCLASS];         // workers of each class that have begun
  Line live[NCLASS];            // workers of each class that have not left
  Line yielded;                 // workers that left early to free their CU
  int64_t cap[NCLASS][NLANE];   // items each lane receives over the graph
  int64_t base[NCLASS][NLANE];  // first ring slot of each lane
  int64_t total[NCLASS];        // items of each class
  int64_t workers[NCLASS];      // workers launched per class
  int64_t watchdog_ticks;       // ticks without progress before giving up
  int64_t yield_ticks;          // idle ticks before a worker may yield its CU
};

// Task metadata word: class, lane, paired items (a work item is two
// consecutive units, as the two halves of a GEMM workgroup take them) and
// the number of items.
DCQ_HD inline uint32_t meta_pack(int cls, int lane, int paired, int64_t items) {
  return (uint32_t)cls | ((uint32_t)lane << 2) | ((uint32_t)(paired ? 1 : 0) << 4) |
         ((uint32_t)items << 8);
}
DCQ_HD inline int meta_class(uint32_t m) { return (int)(m & 3u); }
DCQ_HD inline int meta_lane(uint32_t m) { return (int)((m >> 2) & 3u); }
DCQ_HD inline int meta_step(uint32_t m) { return ((m >> 4) & 1u) ? 2 : 1; }
DCQ_HD inline int64_t meta_items(uint32_t m) { return (int64_t)(m >> 8); }
constexpr int64_t MAX_ITEMS_PER_TASK = (int64_t)1 << 23;

// A ring slot holds (task + 1) << 32 | first unit; 0 marks a slot whose
// item is not written yet.
DCQ_HD inline uint64_t item_enc(int64_t task, int64_t unit) {
  return ((uint64_t)(task + 1) << 32) | (uint64_t)(uint32_t)unit;
}
DCQ_HD inline int64_t item_task(uint64_t it) { return (int64_t)(it >> 32) - 1; }
DCQ_HD inline int item_unit(uint64_t it) { return (int)(uint32_t)(it & 0xffffffffu); }

// Device (or host-model) view of one graph.
struct View {
  Ctl *ctl;
  int32_t *deps;           // per task: predecessors not yet completed
  int32_t *left;           // per task: items not yet completed
  const int32_t *soff;     // CSR successor offsets (ntasks + 1)
  const int32_t *succ;     // CSR successor lists
  const uint32_t *meta;    // per task: meta_pack(...)
  uint64_t *ring;          // every lane's ring, at ctl->base[c][l]
  int32_t *status;         // status[0]: nonzero after a watchdog expiry
};

// Pop results.
constexpr int POP_ITEM = 1, POP_DONE = 0, POP_ABORT = -1;

// Progress watch of one waiting worker.
struct Watch {
  uint64_t seen;   // completed-task count last observed
  uint64_t t0;     // tick at which it was observed
};

template <class AT>
DCQ_HD inline void watch_start(const View &q, Watch &w) {
  w.seen = AT::ld(&q.ctl->completed.v);
  w.t0 = AT::now();
}

// One bounded-wait step: false when the worker must leave (abort seen, or
// no progress for watchdog_ticks, which raises the abort itself).
template <class AT>
DCQ_HD inline bool watch_step(const View &q, Watch &w) {
  Ctl *c = q.ctl;
  if (AT::ld(&c->abort.v)) return false;
  const uint64_t p = AT::ld(&c->completed.v);
  const uint64_t now = AT::now();
  if (p != w.seen) {
    w.seen = p;
    w.t0 = now;
  } else if (now - w.t0 > (uint64_t)c->watchdog_ticks) {
    AT::st(&q.status[0], 1);
    AT::st(&c->abort.v, (uint64_t)1);
    return false;
  }
  AT::pause();
  return true;
}

// A worker's first action.
template <class AT>
DCQ_HD inline void worker_start(const View &q, int cls) {
  AT::add(&q.ctl->started[cls].v, (uint64_t)1);
  AT::add(&q.ctl->live[cls].v, (uint64_t)1);
}

// Leaves early to free the worker's CU if workers of another class have not
// started (see Residency above); false when the worker must stay.
template <class AT>
DCQ_HD inline bool try_yield(const View &q, int cls) {
  Ctl *c = q.ctl;
  int64_t missing = 0;
  for (int k = 0; k < NCLASS; ++k)
    if (k != cls) missing += c->workers[k] - (int64_t)AT::ld(&c->started[k].v);
  uint64_t y = AT::ld(&c->yielded.v);
  while ((int64_t)y < missing)
    if (AT::cas(&c->yielded.v, &y, y + 1)) {
      if (AT::add(&c->live[cls].v, (uint64_t)-1) > 1) return true;
      // the last worker of the class stays
      AT::add(&c->live[cls].v, (uint64_t)1);
      AT::add(&c->yielded.v, (uint64_t)-1);
      return false;
    }
  return false;
}

// Claims the next item of class cls, lanes in order.  Returns POP_ITEM with
// *item set, POP_DONE when every item of the class has been claimed (or the
// worker yielded its CU), or POP_ABORT.  The claimed item's inputs are
// visible to the caller (acquire).
template <class AT>
DCQ_HD inline int pop(const View &q, int cls, uint64_t *item) {
  Ctl *c = q.ctl;
  Watch w;
  watch_start<AT>(q, w);
  const uint64_t idle0 = w.t0;
  for (;;) {
    for (int l = 0; l < NLANE; ++l) {
      if (c->cap[cls][l] == 0) continue;
      uint64_t h = AT::ld(&c->head[cls][l].v);
      while (h < AT::ld(&c->tail[cls][l].v)) {
        if (!AT::cas(&c->head[cls][l].v, &h, h + 1)) continue;   // h was refreshed
        // Slot h is ours.  Its pusher reserved it before writing it, so the
        // item may still be on its way: wait for it (bounded).
        uint64_t *slot = q.ring + c->base[cls][l] + (int64_t)h;
        uint64_t v;
        while ((v = AT::ld(slot)) == 0)
          if (!watch_step<AT>(q, w)) return POP_ABORT;
        AT::fence_acq();
        *item = v;
        return POP_ITEM;
      }
    }
    uint64_t claimed = 0;
    for (int l = 0; l < NLANE; ++l) claimed += AT::ld(&c->head[cls][l].v);
    if ((int64_t)claimed >= c->total[cls]) {
      AT::add(&c->live[cls].v, (uint64_t)-1);
      return POP_DONE;
    }
    if (AT::now() - idle0 > (uint64_t)c->yield_ticks && try_yield<AT>(q, cls)) return POP_DONE;
    if (!watch_step<AT>(q, w)) return POP_ABORT;
  }
}

// Makes every item of task s available: reserves its slots in the ring of
// its class and lane, then writes them.  The caller has issued a release
// fence after the last write the items' consumers must see.
template <class AT>
DCQ_HD inline void push(const View &q, int64_t s) {
  Ctl *c = q.ctl;
  const uint32_t m = q.meta[s];
  const int cls = meta_class(m), lane = meta_lane(m), step = meta_step(m);
  const int64_t n = meta_items(m);
  const uint64_t b = AT::add(&c->tail[cls][lane].v, (uint64_t)n);
  uint64_t *ring = q.ring + c->base[cls][lane] + (int64_t)b;
  for (int64_t i = 0; i < n; ++i) AT::st(&ring[i], item_enc(s, i * step));
}

// Completion of one item of task t.  Precondition: every write of the item
// (by every thread that ran it) is ordered before a release fence that
// precedes this call.  The last item of t releases t's successors; a
// successor whose last predecessor this was is pushed.
template <class AT>
DCQ_HD inline void complete(const View &q, int64_t t) {
  if (AT::add(&q.left[t], -1) != 1) return;
  // every item of t has completed: take the other items' writes along
  // (acquire) and pass them on with this one's through the dependency
  // counters (release)
  AT::fence_acq();
  AT::fence_rel();
  const int32_t j0 = q.soff[t], j1 = q.soff[t + 1];
  bool any = false;
  for (int32_t j = j0; j < j1; ++j) {
    const int32_t s = q.succ[j];
    if (AT::add(&q.deps[s], -1) != 1) continue;
    if (!any) {
      // s's other predecessors completed before: acquire their writes too,
      // then release everything to the workers of the pushed items
      AT::fence_acq();
      AT::fence_rel();
      any = true;
    }
    push<AT>(q, s);
  }
  AT::add(&q.ctl->completed.v, (uint64_t)1);
}

}  // namespace dcq

// Internal host-side state of a dagchol runtime.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <deque>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/dagchol.h"
#include "exec_abi.h"

enum HandleKind { HK_VECTOR = 0, HK_MATRIX = 1 };

// Records a HIP error as the thread's last error message (dc_last_error) and
// returns -EIO.
int dcx_fail_hip(hipError_t e, const char *what);

// Refinement: error left after adding a correction of norm dn whose
// predecessor had norm prev, with the corrections taken to contract
// geometrically at the observed ratio rho = dn / prev:
// rho dn / (1 - rho) = dn^2 / (prev - dn) (the estimate of extra-precise
// iterative refinement, Demmel et al., ACM TOMS 2006).  Only called when
// dn <= prev / 2 (no stagnation), so prev - dn > 0 wherever dn > 0.
inline double dcx_remaining_error(double dn, double prev) {
  return dn > 0 ? dn * dn / (prev - dn) : 0.0;
}

struct Handle {
  int kind = HK_MATRIX;
  void *ptr = nullptr;
  int64_t rows = 0, cols = 0, ld = 1;
  int dtype = DC_F64;
  dc_handle parent = 0;            // 0 for a registered (top-level) handle
  int64_t ti = 0, tj = 0;          // tile coordinates in the parent
  int64_t row_off = 0;             // first row in the top-level matrix
  bool alive = false;
  bool partitioned = false;
  int64_t tile = 0, trows = 0, tcols = 0;
  std::vector<dc_handle> tiles;
  // dependency-inference state for the graph being built
  int64_t last_writer = -1;
  std::vector<int64_t> readers;
  int pending = 0;
  // flushed graphs not yet collected that reference this handle
  int inflight_ref = 0;
  // numerical status of the last factorisation (top-level handles)
  int64_t info = 0;
  // top-level handle whose numerical status this handle's tasks share (0:
  // its own); workspace tiles of a factorisation report into the matrix
  dc_handle status_root = 0;
};

struct Task {
  dcx::TaskDesc desc;
  std::vector<int64_t> preds;
  int64_t nwar = 0;
  int prio = 0;
};

// Fixed buffers for a graph's layout (the calls that may not allocate):
// device memory of cap bytes and a host staging area of the same size.
struct ExtArena {
  void *dev = nullptr;
  void *host = nullptr;
  int64_t cap = 0;
};

// Device and pinned host memory holding one graph's layout.
struct Arena {
  void *dev = nullptr;
  void *host = nullptr;
  int64_t cap = 0;
  bool busy = false;               // a graph in flight uses it
};

// Graphs flushed and not yet collected, at most this many per runtime.
constexpr size_t MAX_INFLIGHT = 8;

// One flushed graph until it is collected.
struct Inflight {
  void *arena_dev = nullptr;       // where the graph's layout lives
  int arena = -1;                  // index in dc_runtime::arenas, -1 for fixed buffers
  int64_t tail_off = 0, tail_bytes = 0, status_off = 0, info_off = 0, trace_off = 0;
  int64_t ntasks = 0;               // tasks laid out (after splitting)
  // first laid-out task of each submitted task (and the total) when some
  // tasks were split, else empty
  std::vector<int64_t> xfirst;
  std::vector<dc_handle> slot_roots;
  std::vector<char> slot_factor;   // slot has a POTRF task in the graph
  std::vector<int32_t> kinds;       // per submitted task
  std::vector<dc_handle> handles;  // handles the flushed graph references
  hipEvent_t done = nullptr;       // recorded after the graph's last launch
  std::vector<hipEvent_t> evs;     // its fork/join events
  // timed launches: (begin event, end event, kernel class, flops, bytes)
  struct Timed { hipEvent_t b, e; int cls; double flops, bytes; };
  std::vector<Timed> timed;
};

struct dc_runtime {
  dc_config cfg{};
  hipStream_t stream = nullptr;
  hipStream_t side = nullptr;                  // panel units next to GEMM units
  hipStream_t side2 = nullptr, side3 = nullptr; // further concurrent worker classes
  std::vector<hipEvent_t> ev_pool;             // free events without timing
  bool ktiming = false;                        // per-kernel timing enabled
  std::vector<hipEvent_t> tev_pool;            // free timing events
  dc_kernel_stats kstats{};
  bool own_stream = false;
  int num_cus = 0;
  int default_workers = 1;
  int wall_clock_khz = 100000;

  std::vector<Handle> handles;                 // id - 1 -> handle
  std::vector<dc_handle> free_ids;             // slots of unregistered handles
  std::unordered_map<void *, dc_handle> by_ptr;
  std::vector<dc_handle> touched;              // handles referenced by pending tasks
  std::vector<Task> tasks;                     // pending graph
  std::unordered_map<dc_handle, int> slot_of;  // root matrix -> status slot
  std::vector<dc_handle> slot_roots;
  std::vector<char> slot_factor;

  void *inv_ws = nullptr;                      // dc_potrf's inverse workspace
  int64_t inv_ws_bytes = 0;
  void *mix_ws = nullptr;                      // dc_potrf's mixed-precision workspace
  int64_t mix_ws_bytes = 0;
  std::vector<Arena> arenas;                   // at most MAX_INFLIGHT
  std::deque<Inflight> flq;                    // flushed graphs, oldest first
  const ExtArena *ext = nullptr;               // set for the duration of a no-alloc call

  std::vector<int64_t> trace_host;
  std::vector<int32_t> trace_kind;
  int64_t trace_t0 = 0;

  double last_build_ms = 0.0;
  int64_t last_units = 0;
  int32_t last_workers = 0;
  int64_t last_levels = 0;
  std::string last_hip_error;

  Handle *get(dc_handle h);
  dc_handle root_of(dc_handle h);
  dc_handle status_root_of(dc_handle h);
  dc_handle new_handle(const Handle &h);
  void free_handle(dc_handle h);
  void reset_graph_state();
};

// Continuous-batching solve server on one GPU.
//
// A request is one SPD system A X = B (A FP64 n x n, lower triangle; B n x r)
// living in device memory.  The server owns a fixed number of slots, each
// with its own runtime (its own HIP streams), and one device memory pool
// from which every admitted request gets its workspace (first fit).  The
// progress call, driven by the caller's loop, never blocks: it advances each
// active request one step when the step's work has finished on the GPU, and
// admits waiting requests in arrival order as soon as a slot and enough pool
// memory are free.  Requests in different slots run concurrently, so the
// work of a newly admitted request overlaps with the requests already on
// the GPU.
//
// Per request (A is only read): factor A (FP64 diagonal tiles;
// off-diagonal tiles FP32 with FP32 or BF16 updates, or all FP64), solve,
// then refine with the FP64 residual r = b - A x until ||d|| <= tol ||x||
// or the contraction estimate of the error left is (per column), or
// stagnation; a breakdown or a failed refinement restarts the
// request with the next wider update precision (BF16 -> FP32 -> FP64).  Every step only submits tasks through
// dc_task_submit and flushes.
#include <errno.h>
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <deque>
#include <map>
#include <vector>

#include "../../include/dagchol.h"
#include "runtime_internal.h"

int dcx_submit_potrs_tiles(dc_runtime *rt, const std::vector<dc_handle> &L, int64_t T,
                           const std::vector<dc_handle> &B, const std::vector<dc_handle> *V,
                           const std::vector<dc_handle> *Y);

namespace {

#define TRY(x) do { int e_ = (x); if (e_) return e_; } while (0)

int submit(dc_runtime *rt, dc_kind k, std::initializer_list<dc_handle> h,
           std::initializer_list<dc_mode> m, int prio, const void *cl = nullptr,
           size_t cls = 0) {
  std::vector<dc_handle> hb(h);
  std::vector<dc_mode> mb(m);
  return dc_task_submit(rt, k, (int)hb.size(), hb.data(), mb.data(), cl, cls, prio);
}

size_t al256(size_t v) { return (v + 255) / 256 * 256; }

// First-fit allocator over [0, size) of one device buffer.
struct Pool {
  size_t size = 0;
  std::map<size_t, size_t> free_;   // offset -> length
  void init(size_t s) { size = s; free_.clear(); free_[0] = s; }
  bool alloc(size_t bytes, size_t *off) {
    bytes = al256(bytes);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        *off = it->first;
        const size_t rest = it->second - bytes;
        const size_t o = it->first + bytes;
        free_.erase(it);
        if (rest) free_[o] = rest;
        return true;
      }
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    bytes = al256(bytes);
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
  size_t largest() const {
    size_t m = 0;
    for (auto &f : free_) m = std::max(m, f.second);
    return m;
  }
};

enum Phase { P_FACTOR, P_SOLVE, P_REFINE, P_FINISH };

struct Request {
  int64_t id = 0;
  int64_t n = 0, r = 0;
  const double *A = nullptr, *B = nullptr;
  double *X = nullptr;
  double arrival = 0.0, admitted = 0.0;
  dc_dtype prec = DC_F32;
  int restarts = 0;
};

struct Slot {
  dc_runtime *rt = nullptr;
  hipEvent_t ev = nullptr;
  bool busy = false;
  Request req;
  Phase phase = P_FACTOR;
  size_t off = 0, bytes = 0;
  // workspace layout (device pointers)
  double *diag = nullptr, *r = nullptr;
  void *w = nullptr, *s = nullptr, *v = nullptr;
  double *y = nullptr;                   // solve scratch (n x r)
  double *hx = nullptr, *hd = nullptr;   // pinned host copies of x and d
  size_t host_cap = 0;
  std::vector<dc_handle> regs;
  dc_handle hA = 0, hB = 0, hX = 0, hR = 0, hW = 0, hS = 0, hV = 0, hVl = 0, hY = 0;
  std::vector<dc_handle> D, Wt, Vall, Yt;
  int64_t T = 0;
  int it = 0;
  std::vector<double> prev;
  double last = 0.0;
  bool converged = false;
};

}  // namespace

struct dc_server {
  dc_server_config cfg{};
  void *pool_ptr = nullptr;
  Pool pool;
  std::vector<Slot> slots;
  std::deque<Request> waiting;
  std::vector<dc_request_result> done;
  int64_t next_id = 1;
  std::chrono::steady_clock::time_point t0;
  double now() const {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
};

namespace {

// Tile size of a request: orders up to whole_max are factored as one tile
// (one POTRF task and one diagonal step per sweep): fewer levels per
// request, but one workgroup carries the whole factorisation; orders from
// large_min use tile_large (larger GEMM units where the request has enough
// tiles to fill the device anyway).
int64_t tile_for(const dc_server_config &c, int64_t n) {
  if (n <= c.whole_max && n >= 1) return n;
  return c.large_min > 0 && n >= c.large_min ? c.tile_large : c.tile;
}

// Panel solves and the diagonal steps of the solves go through the inverses
// of the diagonal factors when every diagonal tile has order >= 16.
bool uses_inverses(int64_t tile, int64_t n) {
  return tile >= 16 && n - (n - 1) / tile * tile >= 16;
}

size_t footprint(const dc_server_config &c, int64_t n, int64_t r, dc_dtype prec) {
  const int64_t tile = tile_for(c, n);
  const int64_t T = (n + tile - 1) / tile;
  size_t b = al256((size_t)T * tile * tile * 8);                // FP64 diagonal tiles
  b += al256((size_t)n * n * (prec == DC_F64 ? 8 : 4));         // off-diagonal tiles
  if (prec == DC_BF16) b += al256((size_t)n * n * 2);           // BF16 copies
  b += al256((size_t)n * r * 8);                                // residual / correction
  if (uses_inverses(tile, n)) {
    b += al256((size_t)T * tile * tile * 8);                    // inverses
    b += al256((size_t)n * r * 8);                              // solve scratch
  }
  return b;
}

int reg(Slot &s, dc_handle *out, void *p, int64_t rows, int64_t cols, int64_t ld, dc_dtype t,
        dc_handle status_root) {
  int e = dc_matrix_register(s.rt, out, p, rows, cols, ld, t);
  if (e) return e;
  s.regs.push_back(*out);
  s.rt->handles[*out - 1].status_root = status_root;
  return 0;
}

void release_slot(dc_server *srv, Slot &s) {
  if (!s.busy) return;
  dc_wait_all(s.rt);
  if (!s.Wt.empty()) dc_matrix_unpartition(s.rt, s.hW);
  s.Wt.clear();
  if (!s.Vall.empty() && s.hV) dc_matrix_unpartition(s.rt, s.hV);
  s.Vall.clear();
  if (!s.Yt.empty()) dc_matrix_unpartition(s.rt, s.hY);
  s.Yt.clear();
  for (auto it = s.regs.rbegin(); it != s.regs.rend(); ++it) dc_unregister(s.rt, *it);
  s.regs.clear();
  s.D.clear();
  srv->pool.release(s.off, s.bytes);
  s.busy = false;
}

void finish(dc_server *srv, Slot &s, int status, int converged) {
  dc_request_result res;
  memset(&res, 0, sizeof(res));
  res.id = s.req.id;
  res.status = status;
  res.converged = converged;
  res.iterations = s.it;
  res.final_prec = s.req.prec;
  res.restarts = s.req.restarts;
  res.last_update = s.last;
  res.arrival = s.req.arrival;
  res.admitted = s.req.admitted;
  res.completed = srv->now();
  if (status == 0) dc_get_info(s.rt, s.hA, &res.info);
  release_slot(srv, s);
  srv->done.push_back(res);
}

// Flushes the slot's pending graph and records the completion event.
int launch(Slot &s) {
  TRY(dc_flush(s.rt));
  return hipEventRecord(s.ev, s.rt->stream) == hipSuccess ? 0 : -EIO;
}

int solve_into(Slot &s, dc_handle V) {
  std::vector<dc_handle> L(s.T * s.T);
  for (int64_t i = 0; i < s.T; ++i)
    for (int64_t j = 0; j < s.T; ++j) L[i * s.T + j] = i == j ? s.D[i] : s.Wt[i * s.T + j];
  const int64_t tile = s.rt->handles[s.hW - 1].tile;
  const int64_t tc = (s.req.r + tile - 1) / tile;
  std::vector<dc_handle> vt(s.T * tc);
  TRY(dc_matrix_partition(s.rt, V, tile, vt.data()));
  std::vector<dc_handle> rows(s.T), yrows(s.T);
  int e = 0;
  for (int64_t j = 0; j < tc && !e; ++j) {
    for (int64_t i = 0; i < s.T; ++i) {
      rows[i] = vt[i * tc + j];
      if (s.v) yrows[i] = s.Yt[i * tc + j];
    }
    e = dcx_submit_potrs_tiles(s.rt, L, s.T, rows, s.v ? &s.Vall : nullptr,
                               s.v ? &yrows : nullptr);
  }
  // the row blocks stay registered until the graph ran; unpartitioning waits
  // for them, so it happens when the step is collected
  return e;
}

// Starts request q on slot s: workspace, copy of A, factor graph.
int start(dc_server *srv, Slot &s, const Request &q, size_t off, size_t bytes) {
  s.busy = true;
  s.req = q;
  s.req.admitted = srv->now();
  s.off = off;
  s.bytes = bytes;
  s.it = 0;
  s.last = 0.0;
  s.converged = false;
  s.prev.assign(q.r, INFINITY);
  const dc_server_config &c = srv->cfg;
  const int64_t n = q.n, r = q.r, tile = tile_for(c, n);
  s.T = (n + tile - 1) / tile;
  char *base = (char *)srv->pool_ptr + off;
  size_t o = 0;
  s.diag = (double *)(base + o); o += al256((size_t)s.T * tile * tile * 8);
  s.w = base + o; o += al256((size_t)n * n * (q.prec == DC_F64 ? 8 : 4));
  s.s = nullptr;
  if (q.prec == DC_BF16) { s.s = base + o; o += al256((size_t)n * n * 2); }
  s.r = (double *)(base + o); o += al256((size_t)n * r * 8);
  // inverses of the diagonal factors: panel solves and the diagonal steps of
  // the solves become MFMA products
  s.v = s.y = nullptr;
  if (uses_inverses(tile, n)) {
    s.v = base + o; o += al256((size_t)s.T * tile * tile * 8);
    s.y = (double *)(base + o);
  }
  if (s.host_cap < (size_t)n * r) {
    if (s.hx) hipHostFree(s.hx);
    if (s.hd) hipHostFree(s.hd);
    s.hx = s.hd = nullptr;
    if (hipHostMalloc((void **)&s.hx, (size_t)n * r * 8, 0) != hipSuccess ||
        hipHostMalloc((void **)&s.hd, (size_t)n * r * 8, 0) != hipSuccess)
      return -ENOMEM;
    s.host_cap = (size_t)n * r;
  }
  // A is only read (by the casts into the factor's tiles and by the residual)
  TRY(reg(s, &s.hA, (void *)q.A, n, n, n, DC_F64, 0));
  TRY(reg(s, &s.hB, (void *)q.B, n, r, r, DC_F64, 0));
  TRY(reg(s, &s.hX, q.X, n, r, r, DC_F64, 0));
  TRY(reg(s, &s.hR, s.r, n, r, r, DC_F64, 0));
  TRY(reg(s, &s.hW, s.w, n, n, n, q.prec == DC_F64 ? DC_F64 : DC_F32, s.hA));
  s.hS = 0;
  if (s.s) TRY(reg(s, &s.hS, s.s, n, n, n, DC_BF16, s.hA));
  s.hV = s.hVl = 0;
  const int64_t last = n - (s.T - 1) * tile;
  if (s.v && s.T > 1) TRY(reg(s, &s.hV, s.v, (s.T - 1) * tile, tile, tile, DC_F64, s.hA));
  if (s.v)
    TRY(reg(s, &s.hVl, (char *)s.v + (size_t)(s.T - 1) * tile * tile * 8, last, last, tile, DC_F64,
            s.hA));
  s.hY = 0;
  if (s.y) TRY(reg(s, &s.hY, s.y, n, r, r, DC_F64, 0));
  s.D.assign(s.T, 0);
  for (int64_t k = 0; k < s.T; ++k) {
    const int64_t nb = std::min(tile, n - k * tile);
    TRY(reg(s, &s.D[k], (char *)s.diag + (size_t)k * tile * tile * 8, nb, nb, tile, DC_F64, s.hA));
  }
  // factor graph
  std::vector<dc_handle> At(s.T * s.T), W(s.T * s.T), S(s.T * s.T, 0),
      V(s.hV ? s.T - 1 : 0);
  TRY(dc_matrix_partition(s.rt, s.hA, tile, At.data()));
  int e = dc_matrix_partition(s.rt, s.hW, tile, W.data());
  if (!e && s.hS) e = dc_matrix_partition(s.rt, s.hS, tile, S.data());
  if (!e && s.hV) e = dc_matrix_partition(s.rt, s.hV, tile, V.data());
  auto a = [&](int64_t i, int64_t j) { return At[i * s.T + j]; };
  auto w = [&](int64_t i, int64_t j) { return W[i * s.T + j]; };
  auto sh = [&](int64_t i, int64_t j) { return S[i * s.T + j]; };
  const bool bf = q.prec == DC_BF16;
  for (int64_t i = 0; i < s.T && !e; ++i) {
    e = submit(s.rt, DC_CAST, {a(i, i), s.D[i]}, {DC_R, DC_W}, 0);
    for (int64_t j = 0; j < i && !e; ++j)
      e = submit(s.rt, DC_CAST, {a(i, j), w(i, j)}, {DC_R, DC_W}, j == 0 ? 0 : 1);
  }
  for (int64_t k = 0; k < s.T && !e; ++k) {
    const int64_t row0 = k * tile;
    e = submit(s.rt, DC_POTRF, {s.D[k]}, {DC_RW}, 0, &row0, sizeof(row0));
    const bool inv = s.hV && k + 1 < s.T;
    if (inv && !e) e = submit(s.rt, DC_TRTRI, {s.D[k], V[k]}, {DC_R, DC_W}, 0);
    for (int64_t i = k + 1; i < s.T && !e; ++i) {
      const int pr = i == k + 1 ? 0 : 1;
      // tile (k+1, k) leads to the next POTRF: substitution, so that TRTRI
      // is not ahead of it on the critical path
      if (inv && i != k + 1)
        e = bf ? submit(s.rt, DC_TRSM_INV_CAST, {s.D[k], V[k], w(i, k), sh(i, k)},
                        {DC_R, DC_R, DC_RW, DC_W}, pr)
               : submit(s.rt, DC_TRSM_INV, {s.D[k], V[k], w(i, k)}, {DC_R, DC_R, DC_RW}, pr);
      else
        e = bf ? submit(s.rt, DC_TRSM_CAST, {s.D[k], w(i, k), sh(i, k)}, {DC_R, DC_RW, DC_W}, pr)
               : submit(s.rt, DC_TRSM, {s.D[k], w(i, k)}, {DC_R, DC_RW}, pr);
    }
    for (int64_t i = k + 1; i < s.T && !e; ++i) {
      const dc_handle xi = bf ? sh(i, k) : w(i, k);
      e = submit(s.rt, DC_SYRK, {xi, s.D[i]}, {DC_R, DC_RW}, i == k + 1 ? 0 : 2);
      for (int64_t j = k + 1; j < i && !e; ++j)
        e = submit(s.rt, DC_GEMM, {xi, bf ? sh(j, k) : w(j, k), w(i, j)}, {DC_R, DC_R, DC_RW},
                   j == k + 1 ? 1 : 2);
    }
  }
  if (!e && s.hVl) e = submit(s.rt, DC_TRTRI, {s.D[s.T - 1], s.hVl}, {DC_R, DC_W}, 0);
  if (!e) e = launch(s);
  if (s.hV) dc_matrix_unpartition(s.rt, s.hV);
  if (s.hS) dc_matrix_unpartition(s.rt, s.hS);
  dc_matrix_unpartition(s.rt, s.hW);
  dc_matrix_unpartition(s.rt, s.hA);
  s.phase = P_FACTOR;
  return e;
}

// Restart with the next wider update precision (BF16 -> FP32 -> FP64) after
// a breakdown or a failed refinement.
void restart_wider(dc_server *srv, Slot &s) {
  Request q = s.req;
  q.prec = q.prec == DC_BF16 ? DC_F32 : DC_F64;
  q.restarts += 1;
  release_slot(srv, s);
  srv->waiting.push_front(q);
}

// Advances slot s whose last step has completed.
int step(dc_server *srv, Slot &s) {
  const dc_server_config &c = srv->cfg;
  const int64_t n = s.req.n, r = s.req.r;
  switch (s.phase) {
    case P_FACTOR: {
      TRY(dc_wait_all(s.rt));   // collects the finished graph and its status
      int64_t info = 0;
      dc_get_info(s.rt, s.hA, &info);
      if (info != 0) {
        if (s.req.prec != DC_F64) { restart_wider(srv, s); return 0; }
        finish(srv, s, 0, 0);
        return 0;
      }
      s.Wt.assign(s.T * s.T, 0);
      const int64_t tile = tile_for(c, n);
      TRY(dc_matrix_partition(s.rt, s.hW, tile, s.Wt.data()));
      if (s.v) {
        s.Vall.assign(s.T, 0);
        if (s.hV) TRY(dc_matrix_partition(s.rt, s.hV, tile, s.Vall.data()));
        s.Vall[s.T - 1] = s.hVl;
        s.Yt.assign(s.T * ((r + tile - 1) / tile), 0);
        TRY(dc_matrix_partition(s.rt, s.hY, tile, s.Yt.data()));
      }
      // x0 = solve(b); then r = b - A x0 and d = solve(r).  Each flush
      // releases the handles it used, so partitions can change between the
      // flushed graphs, which run in stream order.
      TRY(submit(s.rt, DC_CAST, {s.hB, s.hX}, {DC_R, DC_W}, 0));
      TRY(dc_flush(s.rt));
      TRY(solve_into(s, s.hX));
      TRY(dc_flush(s.rt));
      TRY(dc_matrix_unpartition(s.rt, s.hX));
      TRY(submit(s.rt, DC_RESID, {s.hA, s.hX, s.hB, s.hR}, {DC_R, DC_R, DC_R, DC_W}, 0));
      TRY(dc_flush(s.rt));
      TRY(solve_into(s, s.hR));
      TRY(launch(s));
      if (hipMemcpyAsync(s.hd, s.r, (size_t)n * r * 8, hipMemcpyDeviceToHost, s.rt->stream) !=
              hipSuccess ||
          hipMemcpyAsync(s.hx, s.req.X, (size_t)n * r * 8, hipMemcpyDeviceToHost, s.rt->stream) !=
              hipSuccess ||
          hipEventRecord(s.ev, s.rt->stream) != hipSuccess)
        return -EIO;
      s.phase = P_REFINE;
      return 0;
    }
    case P_REFINE: {
      TRY(dc_wait_all(s.rt));
      dc_matrix_unpartition(s.rt, s.hR);
      std::vector<double> dn(r, 0.0), xn(r, 0.0);
      for (int64_t i = 0; i < n; ++i)
        for (int64_t k = 0; k < r; ++k) {
          dn[k] = std::max(dn[k], std::fabs(s.hd[i * r + k]));
          xn[k] = std::max(xn[k], std::fabs(s.hx[i * r + k]));
        }
      bool small = true, grow = false, left_small = s.it > 0;
      s.last = 0.0;
      for (int64_t k = 0; k < r; ++k) {
        if (!(dn[k] <= c.tol * xn[k])) small = false;
        if (s.it > 0 && dn[k] > 0.5 * s.prev[k]) grow = true;
        if (s.it > 0 && !(dcx_remaining_error(dn[k], s.prev[k]) <= c.tol * xn[k]))
          left_small = false;
        s.last = std::max(s.last, xn[k] > 0 ? dn[k] / xn[k] : dn[k]);
      }
      if (grow && !small) {
        if (s.req.prec != DC_F64) { restart_wider(srv, s); return 0; }
        finish(srv, s, 0, 0);
        return 0;
      }
      TRY(submit(s.rt, DC_AXPY, {s.hR, s.hX}, {DC_R, DC_RW}, 0));
      if (small || left_small || s.it + 1 >= c.maxit) {
        TRY(launch(s));
        s.phase = P_FINISH;
        s.converged = small || left_small;
        if (!s.converged) s.it += 1;
        return 0;
      }
      s.prev = dn;
      s.it += 1;
      TRY(dc_flush(s.rt));
      TRY(submit(s.rt, DC_RESID, {s.hA, s.hX, s.hB, s.hR}, {DC_R, DC_R, DC_R, DC_W}, 0));
      TRY(dc_flush(s.rt));
      TRY(solve_into(s, s.hR));
      TRY(launch(s));
      if (hipMemcpyAsync(s.hd, s.r, (size_t)n * r * 8, hipMemcpyDeviceToHost, s.rt->stream) !=
              hipSuccess ||
          hipMemcpyAsync(s.hx, s.req.X, (size_t)n * r * 8, hipMemcpyDeviceToHost, s.rt->stream) !=
              hipSuccess ||
          hipEventRecord(s.ev, s.rt->stream) != hipSuccess)
        return -EIO;
      return 0;
    }
    case P_FINISH: {
      TRY(dc_wait_all(s.rt));
      const bool conv = s.converged;
      if (!conv && s.req.prec != DC_F64) { restart_wider(srv, s); return 0; }
      finish(srv, s, 0, conv ? 1 : 0);
      return 0;
    }
    default:
      return -EINVAL;
  }
}

}  // namespace

extern "C" void dc_server_config_default(dc_server_config *c) {
  if (!c) return;
  memset(c, 0, sizeof(*c));
  c->device = 0;
  c->slots = 4;
  c->pool_bytes = (size_t)64 << 30;
  c->tile = 256;
  c->whole_max = dcx::MAX_TILE;
  c->tile_large = dcx::MAX_TILE;
  c->large_min = 4096;
  c->upd = DC_F32;
  c->tol = 1e-12;
  c->maxit = 30;
}

extern "C" int dc_server_create(dc_server **out, const dc_server_config *cfg) {
  if (!out) return -EINVAL;
  *out = nullptr;
  dc_server_config c;
  if (cfg) c = *cfg; else dc_server_config_default(&c);
  if (c.slots < 1 || c.slots > 64 || c.tile < 1 || c.tile > dcx::MAX_TILE || c.pool_bytes == 0 ||
      c.whole_max < 0 || c.whole_max > dcx::MAX_TILE || c.mixed_min < 0 ||
      c.tile_large < 1 || c.tile_large > dcx::MAX_TILE || c.large_min < 0 ||
      !(c.tol > 0) || c.maxit < 0 || (c.upd != DC_F64 && c.upd != DC_F32 && c.upd != DC_BF16))
    return -EINVAL;
  dc_server *srv = new (std::nothrow) dc_server();
  if (!srv) return -ENOMEM;
  srv->cfg = c;
  srv->t0 = std::chrono::steady_clock::now();
  if (hipSetDevice(c.device) != hipSuccess) { delete srv; return -EIO; }
  if (hipMalloc(&srv->pool_ptr, c.pool_bytes) != hipSuccess) { delete srv; return -ENOMEM; }
  srv->pool.init(c.pool_bytes);
  srv->slots.resize(c.slots);
  for (Slot &s : srv->slots) {
    dc_config rc;
    dc_config_default(&rc);
    rc.device = c.device;
    int e = dc_init(&s.rt, &rc);
    if (!e && hipEventCreateWithFlags(&s.ev, hipEventDisableTiming) != hipSuccess) e = -EIO;
    if (e) { dc_server_destroy(srv); return e; }
  }
  *out = srv;
  return 0;
}

extern "C" int dc_server_destroy(dc_server *srv) {
  if (!srv) return -EINVAL;
  for (Slot &s : srv->slots) {
    if (s.rt) {
      if (s.busy) release_slot(srv, s);
      dc_shutdown(s.rt);
    }
    if (s.ev) hipEventDestroy(s.ev);
    if (s.hx) hipHostFree(s.hx);
    if (s.hd) hipHostFree(s.hd);
  }
  if (srv->pool_ptr) hipFree(srv->pool_ptr);
  delete srv;
  return 0;
}

extern "C" double dc_server_now(dc_server *srv) { return srv ? srv->now() : 0.0; }

extern "C" int dc_server_submit(dc_server *srv, const dc_request *req, int64_t *id) {
  if (!srv || !req || !id || req->n < 1 || req->r < 1 || !req->A || !req->B || !req->X)
    return -EINVAL;
  // low-precision updates only where the factorisation is large enough for
  // them to pay for the extra refinement steps
  const dc_dtype prec = req->n < srv->cfg.mixed_min ? DC_F64 : (dc_dtype)srv->cfg.upd;
  if (footprint(srv->cfg, req->n, req->r, DC_F64) > srv->cfg.pool_bytes) return -ENOMEM;
  Request q;
  q.id = srv->next_id++;
  q.n = req->n;
  q.r = req->r;
  q.A = req->A;
  q.B = req->B;
  q.X = req->X;
  q.arrival = req->arrival;
  q.prec = prec;
  srv->waiting.push_back(q);
  *id = q.id;
  return 0;
}

extern "C" int dc_server_progress(dc_server *srv, dc_request_result *results, int cap, int *ndone,
                                  int *active) {
  if (!srv || !ndone || cap < 0 || (cap > 0 && !results)) return -EINVAL;
  int err = 0;
  // 1. advance requests whose step finished
  for (Slot &s : srv->slots) {
    if (!s.busy) continue;
    const hipError_t q = hipEventQuery(s.ev);
    if (q == hipErrorNotReady) continue;
    if (q != hipSuccess) { err = -EIO; break; }
    int e = step(srv, s);
    if (e) {
      release_slot(srv, s);
      dc_request_result res;
      memset(&res, 0, sizeof(res));
      res.id = s.req.id;
      res.status = e;
      res.arrival = s.req.arrival;
      res.completed = srv->now();
      srv->done.push_back(res);
    }
  }
  // 2. admit waiting requests in arrival order while a slot and memory are free
  while (!err && !srv->waiting.empty()) {
    Slot *free_slot = nullptr;
    for (Slot &s : srv->slots)
      if (!s.busy) { free_slot = &s; break; }
    if (!free_slot) break;
    const Request q = srv->waiting.front();
    const size_t need = footprint(srv->cfg, q.n, q.r, q.prec);
    size_t off;
    if (!srv->pool.alloc(need, &off)) break;
    srv->waiting.pop_front();
    int e = start(srv, *free_slot, q, off, need);
    if (e) {
      release_slot(srv, *free_slot);
      dc_request_result res;
      memset(&res, 0, sizeof(res));
      res.id = q.id;
      res.status = e;
      res.arrival = q.arrival;
      res.completed = srv->now();
      srv->done.push_back(res);
    }
  }
  const int nd = (int)std::min<size_t>(srv->done.size(), (size_t)cap);
  for (int i = 0; i < nd; ++i) results[i] = srv->done[i];
  srv->done.erase(srv->done.begin(), srv->done.begin() + nd);
  *ndone = nd;
  if (active) {
    int a = 0;
    for (Slot &s : srv->slots) a += s.busy ? 1 : 0;
    *active = a + (int)srv->waiting.size();
  }
  return err;
}

// High-level operations of dagchol.  Each one only partitions registered
// matrices and submits tile tasks through dc_task_submit, then waits: they
// are ordinary clients of the task interface (Section 2 of the paper), the
// tiled Cholesky being the partitioning idiom of its Section 5.1.
#include <errno.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "../../include/dagchol.h"
#include "runtime_internal.h"
#include "exec_abi.h"

namespace {

struct Tiles {
  dc_runtime *rt = nullptr;
  dc_handle m = 0;
  int64_t tr = 0, tc = 0;
  std::vector<dc_handle> ids;
  bool active = false;
  int open(dc_runtime *r, dc_handle h, int64_t tile) {
    rt = r;
    m = h;
    Handle *p = rt->get(h);
    if (!p) return -ENOENT;
    tr = (p->rows + tile - 1) / tile;
    tc = (p->cols + tile - 1) / tile;
    ids.assign(tr * tc, 0);
    int e = dc_matrix_partition(rt, h, tile, ids.data());
    active = e == 0;
    return e;
  }
  dc_handle at(int64_t i, int64_t j) const { return ids[i * tc + j]; }
  void close() {
    if (active) dc_matrix_unpartition(rt, m);
    active = false;
  }
  ~Tiles() { close(); }
};

int submit1(dc_runtime *rt, dc_kind k, dc_handle a, dc_mode ma, int prio,
            const void *cl = nullptr, size_t cls = 0) {
  dc_handle b[1] = {a};
  dc_mode m[1] = {ma};
  return dc_task_submit(rt, k, 1, b, m, cl, cls, prio);
}
int submit2(dc_runtime *rt, dc_kind k, dc_handle a, dc_mode ma, dc_handle c, dc_mode mc,
            int prio) {
  dc_handle b[2] = {a, c};
  dc_mode m[2] = {ma, mc};
  return dc_task_submit(rt, k, 2, b, m, nullptr, 0, prio);
}
int submit3(dc_runtime *rt, dc_kind k, dc_handle a, dc_mode ma, dc_handle c, dc_mode mc,
            dc_handle e, dc_mode me, int prio) {
  dc_handle b[3] = {a, c, e};
  dc_mode m[3] = {ma, mc, me};
  return dc_task_submit(rt, k, 3, b, m, nullptr, 0, prio);
}

#define TRY(x) do { int e_ = (x); if (e_) return e_; } while (0)

}  // namespace

// Drops the pending graph without running it (after a failed submission).
void dcx_discard_pending(dc_runtime *rt) {
  rt->reset_graph_state();
  rt->slot_of.clear();
  rt->slot_roots.clear();
  rt->slot_factor.clear();
}

// Right-looking tiled factorisation on partitioned tiles (submission only).
// Priorities (Section 5.3's hints): the diagonal factor, the panel TRSMs and
// the updates of the next panel column come first.  With inverse workspaces
// W (one per diagonal tile but the last), the panel solves of column k are a
// substitution TRSM for tile (k+1, k), and TRTRI(k) followed by
// TRSM_INV(i, k) for i >= k + 2.
int dcx_submit_potrf_tiles(dc_runtime *rt, const std::vector<dc_handle> &A, int64_t T,
                           const std::vector<dc_handle> *W) {
  auto at = [&](int64_t i, int64_t j) { return A[i * T + j]; };
  for (int64_t k = 0; k < T; ++k) {
    TRY(submit1(rt, DC_POTRF, at(k, k), DC_RW, 0));
    if (W && k + 1 < T) {
      // The tile below the diagonal leads to the next POTRF: it is solved by
      // substitution straight from L_kk, so the inversion of L_kk, which
      // only the tiles further down need, runs beside it instead of ahead
      // of it on the critical path.
      TRY(submit2(rt, DC_TRSM, at(k, k), DC_R, at(k + 1, k), DC_RW, 0));
      if (k + 2 < T) {
        TRY(submit2(rt, DC_TRTRI, at(k, k), DC_R, (*W)[k], DC_W, 0));
        for (int64_t i = k + 2; i < T; ++i)
          TRY(submit3(rt, DC_TRSM_INV, at(k, k), DC_R, (*W)[k], DC_R, at(i, k), DC_RW, 1));
      }
    } else {
      for (int64_t i = k + 1; i < T; ++i)
        TRY(submit2(rt, DC_TRSM, at(k, k), DC_R, at(i, k), DC_RW, i == k + 1 ? 0 : 1));
    }
    for (int64_t i = k + 1; i < T; ++i) {
      TRY(submit2(rt, DC_SYRK, at(i, k), DC_R, at(i, i), DC_RW, i == k + 1 ? 0 : 2));
      for (int64_t j = k + 1; j < i; ++j)
        TRY(submit3(rt, DC_GEMM, at(i, k), DC_R, at(j, k), DC_R, at(i, j), DC_RW,
                    j == k + 1 ? 1 : 2));
    }
  }
  return 0;
}

static int submit4(dc_runtime *rt, dc_kind k, dc_handle a, dc_handle c, dc_handle e,
                   dc_handle f, int prio) {
  dc_handle b[4] = {a, c, e, f};
  dc_mode m[4] = {DC_R, DC_R, DC_R, DC_W};
  return dc_task_submit(rt, k, 4, b, m, nullptr, 0, prio);
}

// Forward then backward sweep on partitioned L tiles and RHS row blocks.
// With V (the inverses of all diagonal factors) and Y (row blocks of a
// scratch of B's shape) the diagonal steps are out-of-place products with
// the inverses: forward B_k -> Y_k with the updates reading Y_k, backward
// Y_k -> B_k with the updates of Y_i reading B_k; the solution ends in B.
int dcx_submit_potrs_tiles(dc_runtime *rt, const std::vector<dc_handle> &L, int64_t T,
                           const std::vector<dc_handle> &B, const std::vector<dc_handle> *V,
                           const std::vector<dc_handle> *Y) {
  auto at = [&](int64_t i, int64_t j) { return L[i * T + j]; };
  if (V && Y) {
    for (int64_t k = 0; k < T; ++k) {
      TRY(submit4(rt, DC_TRSM_L_INV, at(k, k), (*V)[k], B[k], (*Y)[k], 0));
      for (int64_t i = k + 1; i < T; ++i)
        TRY(submit3(rt, DC_GEMM_RHS_N, at(i, k), DC_R, (*Y)[k], DC_R, B[i], DC_RW,
                    i == k + 1 ? 0 : 1));
    }
    for (int64_t k = T - 1; k >= 0; --k) {
      TRY(submit4(rt, DC_TRSM_LT_INV, at(k, k), (*V)[k], (*Y)[k], B[k], 0));
      for (int64_t i = k - 1; i >= 0; --i)
        TRY(submit3(rt, DC_GEMM_RHS_T, at(k, i), DC_R, B[k], DC_R, (*Y)[i], DC_RW,
                    i == k - 1 ? 0 : 1));
    }
    return 0;
  }
  for (int64_t k = 0; k < T; ++k) {
    TRY(submit2(rt, DC_TRSM_L, at(k, k), DC_R, B[k], DC_RW, 0));
    for (int64_t i = k + 1; i < T; ++i)
      TRY(submit3(rt, DC_GEMM_RHS_N, at(i, k), DC_R, B[k], DC_R, B[i], DC_RW, i == k + 1 ? 0 : 1));
  }
  for (int64_t k = T - 1; k >= 0; --k) {
    TRY(submit2(rt, DC_TRSM_LT, at(k, k), DC_R, B[k], DC_RW, 0));
    for (int64_t i = k - 1; i >= 0; --i)
      TRY(submit3(rt, DC_GEMM_RHS_T, at(k, i), DC_R, B[k], DC_R, B[i], DC_RW, i == k - 1 ? 0 : 1));
  }
  return 0;
}

// Order of the last diagonal tile.
static int64_t last_tile_order(int64_t n, int64_t tile) { return n - (n - 1) / tile * tile; }

// Grows the runtime's inverse workspace to at least `bytes`; the previous
// contents are not kept.
static int inv_workspace(dc_runtime *rt, int64_t bytes) {
  if (rt->inv_ws_bytes >= bytes) return 0;
  if (rt->inv_ws) {
    if (hipStreamSynchronize(rt->stream) != hipSuccess) return -EIO;
    hipFree(rt->inv_ws);
    rt->inv_ws = nullptr;
    rt->inv_ws_bytes = 0;
  }
  if (hipMalloc(&rt->inv_ws, bytes) != hipSuccess) {
    rt->inv_ws = nullptr;
    return -ENOMEM;
  }
  rt->inv_ws_bytes = bytes;
  return 0;
}

int dcx_submit_mixed_factor(dc_runtime *rt, int64_t T, int64_t tile,
                            const std::vector<dc_handle> &At, const std::vector<dc_handle> &D,
                            const std::vector<dc_handle> &W, const std::vector<dc_handle> &S,
                            dc_dtype upd, const std::vector<dc_handle> *V);

// Grows the runtime's mixed-precision factor workspace to at least `bytes`.
static int mix_workspace(dc_runtime *rt, int64_t bytes) {
  if (rt->mix_ws_bytes >= bytes) return 0;
  if (rt->mix_ws) {
    if (hipStreamSynchronize(rt->stream) != hipSuccess) return -EIO;
    hipFree(rt->mix_ws);
    rt->mix_ws = nullptr;
    rt->mix_ws_bytes = 0;
  }
  if (hipMalloc(&rt->mix_ws, bytes) != hipSuccess) {
    rt->mix_ws = nullptr;
    return -ENOMEM;
  }
  rt->mix_ws_bytes = bytes;
  return 0;
}

// The factorisation with low-precision trailing updates, in place in A:
// diagonal tiles factored in A (FP64 POTRF), off-diagonal tiles copied to
// FP32 (plus BF16 copies for upd == BF16), factored there with the mixed
// updates, and copied back into A (exactly: FP32 values are FP64 values).
static int potrf_mixed(dc_runtime *rt, dc_handle A, int64_t n, int64_t tile, dc_dtype upd) {
  const int64_t T = (n + tile - 1) / tile;
  const bool inv = tile >= 16 && T > 1;
  auto al = [](int64_t v) { return (v + 255) / 256 * 256; };
  const int64_t o_w = 0;
  const int64_t o_s = al(o_w + n * n * 4);
  const int64_t o_v = al(o_s + (upd == DC_BF16 ? n * n * 2 : 0));
  const int64_t total = al(o_v + (inv ? (T - 1) * tile * tile * 8 : 0));
  TRY(mix_workspace(rt, total));
  char *base = (char *)rt->mix_ws;
  std::vector<dc_handle> regs;
  auto reg = [&](dc_handle *h, void *ptr, int64_t rows, int64_t cols, int64_t ld, dc_dtype t) {
    int e = dc_matrix_register(rt, h, ptr, rows, cols, ld, t);
    if (e) return e;
    regs.push_back(*h);
    rt->handles[*h - 1].status_root = A;   // workspace tasks report into A's status
    return 0;
  };
  dc_handle hW = 0, hS = 0, hV = 0;
  int e = reg(&hW, base + o_w, n, n, n, DC_F32);
  if (!e && upd == DC_BF16) e = reg(&hS, base + o_s, n, n, n, DC_BF16);
  if (!e && inv) e = reg(&hV, base + o_v, (T - 1) * tile, tile, tile, DC_F64);
  {
    Tiles ta, tw, ts, tv;
    if (!e) e = ta.open(rt, A, tile);
    if (!e) e = tw.open(rt, hW, tile);
    if (!e && hS) e = ts.open(rt, hS, tile);
    if (!e && hV) e = tv.open(rt, hV, tile);
    if (!e) {
      std::vector<dc_handle> D(T), S(T * T, 0), V;
      for (int64_t k = 0; k < T; ++k) D[k] = ta.at(k, k);
      if (hS) S = ts.ids;
      if (hV) for (int64_t k = 0; k + 1 < T; ++k) V.push_back(tv.at(k, 0));
      e = dcx_submit_mixed_factor(rt, T, tile, ta.ids, D, tw.ids, S, upd, hV ? &V : nullptr);
      for (int64_t i = 1; i < T && !e; ++i)
        for (int64_t j = 0; j < i && !e; ++j)
          e = submit2(rt, DC_CAST, tw.at(i, j), DC_R, ta.at(i, j), DC_W, 2);
      if (e) dcx_discard_pending(rt);
      else e = dc_wait_all(rt);
    }
  }
  for (auto it = regs.rbegin(); it != regs.rend(); ++it) {
    const int e2 = dc_unregister(rt, *it);
    if (!e) e = e2;
  }
  return e;
}

extern "C" int dc_potrf(dc_runtime *rt, dc_handle A, int64_t tile, dc_dtype upd) {
  if (!rt) return -EINVAL;
  Handle *p = rt->get(A);
  if (!p) return -ENOENT;
  if (p->rows != p->cols || p->dtype != DC_F64 || tile < 1 || tile > dcx::MAX_TILE ||
      (upd != DC_F64 && upd != DC_F32 && upd != DC_BF16))
    return -EINVAL;
  if (p->partitioned) return -EBUSY;
  if (p->rows == 0) { p->info = 0; return 0; }
  if (upd != DC_F64) {
    if (rt->cfg.device < 0) return -ENODEV;
    return potrf_mixed(rt, A, p->rows, tile, upd);
  }
  const int64_t n = p->rows;
  const int64_t T = (n + tile - 1) / tile;
  // inverse workspaces: tiles - 1 full diagonal tiles, kept by the runtime
  const bool inv = tile >= 16 && T > 1 && rt->cfg.device >= 0;
  dc_handle wh = 0;
  Tiles tw;
  if (inv) {
    TRY(inv_workspace(rt, (T - 1) * tile * tile * 8));
    TRY(dc_matrix_register(rt, &wh, rt->inv_ws, (T - 1) * tile, tile, tile, DC_F64));
    const int e = tw.open(rt, wh, tile);
    if (e) { dc_unregister(rt, wh); return e; }
  }
  int e;
  {
    Tiles t;
    e = t.open(rt, A, tile);
    if (!e) {
      e = dcx_submit_potrf_tiles(rt, t.ids, t.tr, inv ? &tw.ids : nullptr);
      if (e) dcx_discard_pending(rt);
      else e = dc_wait_all(rt);
    }
  }
  if (inv) {
    tw.close();
    const int e2 = dc_unregister(rt, wh);
    if (!e) e = e2;
  }
  return e;
}

extern "C" int dc_potrf_noalloc(dc_runtime *rt, dc_handle A, int64_t tile) {
  if (!rt) return -EINVAL;
  Handle *p = rt->get(A);
  if (!p) return -ENOENT;
  if (p->rows != p->cols || p->dtype != DC_F64 || tile < 1 || tile > dcx::MAX_TILE)
    return -EINVAL;
  if (p->partitioned) return -EBUSY;
  if (rt->cfg.device < 0) return -ENODEV;
  if (p->rows == 0) { p->info = 0; return 0; }
  ExtArena arena;
  if (dcx_noalloc_scratch(rt->cfg.device, &arena.dev, &arena.host, &arena.cap)) return -EIO;
  // a graph flushed before this call runs on the runtime's own arena
  TRY(dc_wait_all(rt));
  int e;
  {
    Tiles t;
    e = t.open(rt, A, tile);
    if (!e) {
      // panel solves by substitution: no inverse workspace
      e = dcx_submit_potrf_tiles(rt, t.ids, t.tr, nullptr);
      if (e) {
        dcx_discard_pending(rt);
      } else {
        const bool timing = rt->ktiming;
        rt->ktiming = false;   // timing events would be created on demand
        rt->ext = &arena;
        e = dc_wait_all(rt);
        rt->ext = nullptr;
        rt->ktiming = timing;
      }
    }
  }
  return e;
}

extern "C" int dc_potrs(dc_runtime *rt, dc_handle L, dc_handle B, int64_t tile) {
  if (!rt) return -EINVAL;
  Handle *pl = rt->get(L);
  Handle *pb = rt->get(B);
  if (!pl || !pb) return -ENOENT;
  if (pl->rows != pl->cols || pb->rows != pl->rows || pb->dtype != DC_F64 ||
      pl->dtype != DC_F64 || tile < 1 || tile > dcx::MAX_TILE)
    return -EINVAL;
  if (pl->partitioned || pb->partitioned) return -EBUSY;
  if (pl->rows == 0 || pb->cols == 0) return 0;
  const int64_t n = pl->rows;
  const int64_t T = (n + tile - 1) / tile;
  const int64_t last = n - (T - 1) * tile;
  // inverses of the diagonal factors (all of order >= 16): TRTRI for all of
  // them first, in parallel, then out-of-place products instead of the
  // diagonal substitutions of both sweeps, through a scratch Y of B's shape
  const int64_t r = pb->cols;
  const bool inv = tile >= 16 && last_tile_order(n, tile) >= 16 && rt->cfg.device >= 0;
  dc_handle hw = 0, hl = 0, hy = 0;
  Tiles tw, ty;
  std::vector<dc_handle> V;
  int e = 0;
  if (inv) {
    const int64_t wbytes = T * tile * tile * 8;
    TRY(inv_workspace(rt, wbytes + n * r * 8));
    TRY(dc_matrix_register(rt, &hy, (char *)rt->inv_ws + wbytes, n, r, r, DC_F64));
    e = ty.open(rt, hy, tile);
    V.assign(T, 0);
    if (T > 1 && !e) {
      e = dc_matrix_register(rt, &hw, rt->inv_ws, (T - 1) * tile, tile, tile, DC_F64);
      if (!e) e = tw.open(rt, hw, tile);
      for (int64_t k = 0; k + 1 < T && !e; ++k) V[k] = tw.at(k, 0);
    }
    if (!e && last >= 16)
      e = dc_matrix_register(rt, &hl, (char *)rt->inv_ws + (T - 1) * tile * tile * 8, last, last,
                             tile, DC_F64);
    if (!e && hl) V[T - 1] = hl;
  }
  if (!e) {
    Tiles tl, tb;
    e = tl.open(rt, L, tile);
    if (!e) e = tb.open(rt, B, tile);
    for (int64_t k = 0; k < T && inv && !e; ++k)
      if (V[k]) e = submit2(rt, DC_TRTRI, tl.at(k, k), DC_R, V[k], DC_W, 0);
    // each column block of B is an independent right-hand-side group
    std::vector<dc_handle> rows(tl.tr), yrows(tl.tr);
    for (int64_t j = 0; j < tb.tc && !e; ++j) {
      for (int64_t i = 0; i < tl.tr; ++i) {
        rows[i] = tb.at(i, j);
        if (inv) yrows[i] = ty.at(i, j);
      }
      e = dcx_submit_potrs_tiles(rt, tl.ids, tl.tr, rows, inv ? &V : nullptr,
                                 inv ? &yrows : nullptr);
    }
    if (e) dcx_discard_pending(rt);
    else e = dc_wait_all(rt);
  }
  tw.close();
  ty.close();
  for (dc_handle h : {hw, hl, hy})
    if (h) { const int e2 = dc_unregister(rt, h); if (!e) e = e2; }
  return e;
}

// Many independent factorisations (and solves) in one graph: one flush, one
// set of level launches for the whole batch.  tiles[i] == 0 selects the
// matrix order (a single POTRF task); B[i] == 0 skips the solve.
extern "C" int dc_potrf_batched(dc_runtime *rt, int64_t count, const dc_handle *A,
                                const dc_handle *B, const int64_t *tiles, int64_t *info_out) {
  if (!rt || count < 0 || (count > 0 && (!A || !tiles))) return -EINVAL;
  for (int64_t i = 0; i < count; ++i) {
    Handle *p = rt->get(A[i]);
    if (!p) return -ENOENT;
    const int64_t tile = tiles[i] > 0 ? std::min(tiles[i], p->rows) : p->rows;
    // FP32 matrices are factored as one tile (POTRF on FP32 storage)
    if (p->rows != p->cols || (p->dtype != DC_F64 && p->dtype != DC_F32) || tiles[i] < 0 ||
        (p->rows > 0 && (tile < 1 || tile > dcx::MAX_TILE)) ||
        (p->dtype == DC_F32 && tile < p->rows))
      return -EINVAL;
    if (p->partitioned) return -EBUSY;
    if (B && B[i]) {
      Handle *q = rt->get(B[i]);
      if (!q) return -ENOENT;
      if (q->rows != p->rows || q->dtype != DC_F64) return -EINVAL;
      if (q->partitioned) return -EBUSY;
    }
  }
  int err = dc_wait_all(rt);
  if (err) return err;
  std::vector<Tiles> ta(count), tb(count);
  for (int64_t i = 0; i < count && !err; ++i) {
    Handle *p = rt->get(A[i]);
    if (p->rows == 0) continue;
    const int64_t tile = tiles[i] > 0 ? std::min<int64_t>(tiles[i], p->rows) : p->rows;
    if (tile == p->rows) {
      // one tile: the tasks take the registered handles themselves (no
      // partition to create and undo)
      const dc_handle a1[1] = {A[i]};
      const std::vector<dc_handle> ids(a1, a1 + 1);
      err = dcx_submit_potrf_tiles(rt, ids, 1, nullptr);
      if (!err && B && B[i] && rt->get(B[i])->cols > 0) {
        const std::vector<dc_handle> rows(1, B[i]);
        err = dcx_submit_potrs_tiles(rt, ids, 1, rows, nullptr, nullptr);
      }
      continue;
    }
    err = ta[i].open(rt, A[i], tile);
    if (!err) err = dcx_submit_potrf_tiles(rt, ta[i].ids, ta[i].tr, nullptr);
    if (!err && B && B[i] && rt->get(B[i])->cols > 0) {
      err = tb[i].open(rt, B[i], tile);
      std::vector<dc_handle> rows(ta[i].tr);
      for (int64_t j = 0; j < tb[i].tc && !err; ++j) {
        for (int64_t r = 0; r < ta[i].tr; ++r) rows[r] = tb[i].at(r, j);
        err = dcx_submit_potrs_tiles(rt, ta[i].ids, ta[i].tr, rows, nullptr, nullptr);
      }
    }
  }
  if (err) {
    dcx_discard_pending(rt);
    return err;
  }
  err = dc_wait_all(rt);
  if (info_out)
    for (int64_t i = 0; i < count; ++i) dc_get_info(rt, A[i], &info_out[i]);
  return err;
}

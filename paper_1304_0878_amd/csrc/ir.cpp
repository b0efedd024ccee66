// Mixed-precision Cholesky solve with FP64-residual iterative refinement.
//
// Only submits tasks through dc_task_submit and waits.  The factor is kept
// in a runtime-owned workspace: the diagonal tiles in FP64 (POTRF stays
// FP64), the off-diagonal tiles in FP32 and, for BF16 updates, a BF16 copy
// of each finished panel tile written by the TRSM.  A stays untouched and is
// the matrix of the FP64 residual r = b - A x.
#include <errno.h>
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <vector>

#include "../../include/dagchol.h"
#include "runtime_internal.h"

int dcx_submit_potrf_tiles(dc_runtime *rt, const std::vector<dc_handle> &A, int64_t T,
                           const std::vector<dc_handle> *W);
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

// Copies an n x r row-major device matrix with leading dimension ld into a
// dense host array; strided copies go in blocks of rows (rectangular copies
// of very many rows are not accepted by the runtime).
hipError_t copy_rows_to_host(double *dst, const double *src, int64_t ld, int64_t n, int64_t r) {
  if (ld == r) return hipMemcpy(dst, src, (size_t)n * r * 8, hipMemcpyDeviceToHost);
  for (int64_t i0 = 0; i0 < n; i0 += 4096) {
    const int64_t rows = std::min<int64_t>(4096, n - i0);
    const hipError_t e = hipMemcpy2D(dst + i0 * r, r * 8, src + i0 * ld, ld * 8, r * 8, rows,
                                     hipMemcpyDeviceToHost);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

struct Scratch {
  void *ptr = nullptr;
  size_t bytes = 0;
  ~Scratch() { if (ptr) hipFree(ptr); }
  int get(size_t b) {
    if (b <= bytes) return 0;
    if (ptr) hipFree(ptr);
    ptr = nullptr;
    bytes = 0;
    if (hipMalloc(&ptr, b) != hipSuccess) { ptr = nullptr; return -ENOMEM; }
    bytes = b;
    return 0;
  }
};

// Handles registered for one call; all unregistered on scope exit.
struct Regs {
  dc_runtime *rt;
  std::vector<dc_handle> hs;
  explicit Regs(dc_runtime *r) : rt(r) {}
  int mat(dc_handle *out, void *p, int64_t rows, int64_t cols, int64_t ld, dc_dtype t,
          dc_handle status_root) {
    int e = dc_matrix_register(rt, out, p, rows, cols, ld, t);
    if (e) return e;
    hs.push_back(*out);
    rt->handles[*out - 1].status_root = status_root;
    return 0;
  }
  ~Regs() {
    for (auto it = hs.rbegin(); it != hs.rend(); ++it) dc_unregister(rt, *it);
  }
};

double now_ms() {
  return std::chrono::duration<double, std::milli>(
             std::chrono::steady_clock::now().time_since_epoch()).count();
}

}  // namespace

// Submits the factorisation of A (FP64 lower, partitioned tiles At) at update
// precision upd into the workspace: D[k] FP64 diagonal tiles, W (FP32) and S
// (BF16) off-diagonal tile handles.  For upd == FP64 the tiles W are FP64.
// With V (T - 1 FP64 tiles), the panel solves of column k are TRTRI(D[k])
// into V[k] and TRSM_INV (TRSM_INV_CAST for BF16) instead of TRSM, except
// for tile (k+1, k): it leads to the next POTRF and is solved by
// substitution, so TRTRI runs beside it rather than ahead of it.  When D[k]
// is A's own diagonal tile (factored in place) no copy is made.
int dcx_submit_mixed_factor(dc_runtime *rt, int64_t T, int64_t tile,
                            const std::vector<dc_handle> &At, const std::vector<dc_handle> &D,
                            const std::vector<dc_handle> &W, const std::vector<dc_handle> &S,
                            dc_dtype upd, const std::vector<dc_handle> *V) {
  auto a = [&](int64_t i, int64_t j) { return At[i * T + j]; };
  auto w = [&](int64_t i, int64_t j) { return W[i * T + j]; };
  auto s = [&](int64_t i, int64_t j) { return S[i * T + j]; };
  for (int64_t i = 0; i < T; ++i) {
    if (D[i] != a(i, i)) TRY(submit(rt, DC_CAST, {a(i, i), D[i]}, {DC_R, DC_W}, 0));
    for (int64_t j = 0; j < i; ++j)
      TRY(submit(rt, DC_CAST, {a(i, j), w(i, j)}, {DC_R, DC_W}, j == 0 ? 0 : 1));
  }
  const bool bf = upd == DC_BF16;
  for (int64_t k = 0; k < T; ++k) {
    const int64_t row0 = k * tile;
    TRY(submit(rt, DC_POTRF, {D[k]}, {DC_RW}, 0, &row0, sizeof(row0)));
    const bool inv = V && k + 1 < T;
    if (inv) TRY(submit(rt, DC_TRTRI, {D[k], (*V)[k]}, {DC_R, DC_W}, 0));
    for (int64_t i = k + 1; i < T; ++i) {
      const int pr = i == k + 1 ? 0 : 1;
      const bool inv_i = inv && i != k + 1;
      if (inv_i && bf)
        TRY(submit(rt, DC_TRSM_INV_CAST, {D[k], (*V)[k], w(i, k), s(i, k)},
                   {DC_R, DC_R, DC_RW, DC_W}, pr));
      else if (inv_i)
        TRY(submit(rt, DC_TRSM_INV, {D[k], (*V)[k], w(i, k)}, {DC_R, DC_R, DC_RW}, pr));
      else if (bf)
        TRY(submit(rt, DC_TRSM_CAST, {D[k], w(i, k), s(i, k)}, {DC_R, DC_RW, DC_W}, pr));
      else
        TRY(submit(rt, DC_TRSM, {D[k], w(i, k)}, {DC_R, DC_RW}, pr));
    }
    for (int64_t i = k + 1; i < T; ++i) {
      const dc_handle xi = bf ? s(i, k) : w(i, k);
      TRY(submit(rt, DC_SYRK, {xi, D[i]}, {DC_R, DC_RW}, i == k + 1 ? 0 : 2));
      for (int64_t j = k + 1; j < i; ++j) {
        const dc_handle xj = bf ? s(j, k) : w(j, k);
        TRY(submit(rt, DC_GEMM, {xi, xj, w(i, j)}, {DC_R, DC_R, DC_RW}, j == k + 1 ? 1 : 2));
      }
    }
  }
  return 0;
}

extern "C" int dc_posv_ir(dc_runtime *rt, dc_handle A, dc_handle B, dc_handle X, int64_t tile,
                          dc_dtype upd, double tol, int maxit, dc_ir_report *rep) {
  if (!rt) return -EINVAL;
  if (rt->cfg.device < 0) return -ENODEV;
  Handle *pa = rt->get(A), *pb = rt->get(B), *px = rt->get(X);
  if (!pa || !pb || !px) return -ENOENT;
  const int64_t n = pa->rows, r = pb->cols;
  if (pa->cols != n || pa->dtype != DC_F64 || pb->dtype != DC_F64 || px->dtype != DC_F64 ||
      pb->rows != n || px->rows != n || px->cols != r || tile < 1 || tile > dcx::MAX_TILE ||
      !(tol > 0) || maxit < 0 || (upd != DC_F64 && upd != DC_F32 && upd != DC_BF16))
    return -EINVAL;
  if (pa->partitioned || pb->partitioned || px->partitioned) return -EBUSY;
  // registering the workspace below may move the handle storage: keep what
  // is needed of X, and do not use the handle pointers afterwards
  const double *const xptr = (const double *)px->ptr;
  const int64_t xld = px->ld;
  pa = pb = px = nullptr;
  dc_ir_report local;
  memset(&local, 0, sizeof(local));
  if (!rep) rep = &local;
  memset(rep, 0, sizeof(*rep));
  if (n == 0 || r == 0) { rep->converged = 1; return 0; }
  TRY(dc_wait_all(rt));

  const int64_t T = (n + tile - 1) / tile;
  // workspace: diagonal tiles | off-diagonal FP32 or FP64 | BF16 copies | R
  auto al = [](size_t v) { return (v + 255) / 256 * 256; };
  Scratch ws;
  std::vector<double> hx((size_t)n * r), hd((size_t)n * r);

  dc_dtype prec = upd;
  for (;;) {
    const size_t es = prec == DC_F64 ? 8 : 4;
    const size_t o_d = 0;
    const size_t o_w = al(o_d + (size_t)T * tile * tile * 8);
    const size_t o_s = al(o_w + (size_t)n * n * es);
    const size_t o_r = al(o_s + (prec == DC_BF16 ? (size_t)n * n * 2 : 0));
    // inverses of the diagonal factors: panel solves and the diagonal steps
    // of every solve become MFMA products
    const int64_t nlast = n - (T - 1) * tile;
    const bool inv = tile >= 16 && nlast >= 16;
    const size_t o_v = al(o_r + (size_t)n * r * 8);
    const size_t o_y = al(o_v + (inv ? (size_t)T * tile * tile * 8 : 0));   // solve scratch
    const size_t total = al(o_y + (inv ? (size_t)n * r * 8 : 0));
    TRY(ws.get(total));
    char *base = (char *)ws.ptr;
    Regs regs(rt);
    dc_handle hW, hS = 0, hR;
    TRY(regs.mat(&hW, base + o_w, n, n, n, prec == DC_F64 ? DC_F64 : DC_F32, A));
    if (prec == DC_BF16) TRY(regs.mat(&hS, base + o_s, n, n, n, DC_BF16, A));
    TRY(regs.mat(&hR, base + o_r, n, r, r, DC_F64, 0));
    dc_handle hV = 0, hVl = 0, hY = 0;   // inverse tiles 0..T-2 and T-1; solve scratch
    if (inv) TRY(regs.mat(&hY, base + o_y, n, r, r, DC_F64, 0));
    if (inv && T > 1) TRY(regs.mat(&hV, base + o_v, (T - 1) * tile, tile, tile, DC_F64, A));
    if (inv && nlast >= 16)
      TRY(regs.mat(&hVl, base + o_v + (size_t)(T - 1) * tile * tile * 8, nlast, nlast, tile,
                   DC_F64, A));
    std::vector<dc_handle> D(T);
    for (int64_t k = 0; k < T; ++k) {
      const int64_t nb = std::min(tile, n - k * tile);
      TRY(regs.mat(&D[k], base + o_d + (size_t)k * tile * tile * 8, nb, nb, tile, DC_F64, A));
    }

    // ---- factor
    double t0 = now_ms();
    int64_t info = 0;
    {
      std::vector<dc_handle> At(T * T), W(T * T), S(T * T, 0), V(inv ? T - 1 : 0);
      TRY(dc_matrix_partition(rt, A, tile, At.data()));
      int e = dc_matrix_partition(rt, hW, tile, W.data());
      if (!e && hS) e = dc_matrix_partition(rt, hS, tile, S.data());
      if (!e && hV) e = dc_matrix_partition(rt, hV, tile, V.data());
      if (!e) e = dcx_submit_mixed_factor(rt, T, tile, At, D, W, S, prec, hV ? &V : nullptr);
      if (!e && hVl) e = submit(rt, DC_TRTRI, {D[T - 1], hVl}, {DC_R, DC_W}, 0);
      if (!e) e = dc_wait_all(rt);
      if (hV) dc_matrix_unpartition(rt, hV);
      if (hS) dc_matrix_unpartition(rt, hS);
      dc_matrix_unpartition(rt, hW);
      dc_matrix_unpartition(rt, A);
      TRY(e);
      TRY(dc_get_info(rt, A, &info));
    }
    rep->factor_ms = now_ms() - t0;
    if (info != 0) {
      if (prec == DC_F64) { rep->final_prec = DC_F64; return 0; }   // A not SPD: info set
      prec = prec == DC_BF16 ? DC_F32 : DC_F64;
      rep->fallbacks++;
      continue;
    }

    // ---- solve and refine
    double t1 = now_ms();
    std::vector<dc_handle> Wt(T * T), L(T * T), Xb, Rb, Vall;
    TRY(dc_matrix_partition(rt, hW, tile, Wt.data()));
    if (inv) {
      Vall.assign(T, 0);
      if (hV) TRY(dc_matrix_partition(rt, hV, tile, Vall.data()));
      Vall[T - 1] = hVl;
    }
    for (int64_t i = 0; i < T; ++i)
      for (int64_t j = 0; j < T; ++j) L[i * T + j] = i == j ? D[i] : Wt[i * T + j];
    auto solve_into = [&](dc_handle V) -> int {
      // V (n x r) is solved in place with the mixed factor (through the
      // scratch Y when the inverses are there)
      const int64_t tc = (r + tile - 1) / tile;
      std::vector<dc_handle> vt(T * tc), yt(T * tc);
      TRY(dc_matrix_partition(rt, V, tile, vt.data()));
      int e = inv ? dc_matrix_partition(rt, hY, tile, yt.data()) : 0;
      std::vector<dc_handle> rows(T), yrows(T);
      for (int64_t j = 0; j < tc && !e; ++j) {
        for (int64_t i = 0; i < T; ++i) {
          rows[i] = vt[i * tc + j];
          yrows[i] = yt[i * tc + j];
        }
        e = dcx_submit_potrs_tiles(rt, L, T, rows, inv ? &Vall : nullptr, inv ? &yrows : nullptr);
      }
      if (!e) e = dc_wait_all(rt);
      if (inv) dc_matrix_unpartition(rt, hY);
      dc_matrix_unpartition(rt, V);
      return e;
    };
    int e = submit(rt, DC_CAST, {B, X}, {DC_R, DC_W}, 0);
    if (!e) e = dc_wait_all(rt);
    if (!e) e = solve_into(X);
    std::vector<double> prev(r, INFINITY), xn(r), dn(r);
    int it = 0;
    bool converged = false;
    double last = 0.0;
    auto colmax = [&](const std::vector<double> &v, std::vector<double> &out) {
      std::fill(out.begin(), out.end(), 0.0);
      for (int64_t i = 0; i < n; ++i)
        for (int64_t c = 0; c < r; ++c) out[c] = std::max(out[c], std::fabs(v[i * r + c]));
    };
    while (!e) {
      // r = b - A x (compensated), d = solve(r)
      e = submit(rt, DC_RESID, {A, X, B, hR}, {DC_R, DC_R, DC_R, DC_W}, 0);
      if (!e) e = dc_wait_all(rt);
      if (!e) e = solve_into(hR);
      if (e) break;
      hipError_t he = hipGetLastError();
      if (he != hipSuccess) {
        e = dcx_fail_hip(he, "error pending before the refinement copies");
        break;
      }
      he = hipMemcpy(hd.data(), base + o_r, hd.size() * 8, hipMemcpyDeviceToHost);
      if (he != hipSuccess) {
        e = dcx_fail_hip(he, "copy of the correction to the host");
        break;
      }
      he = copy_rows_to_host(hx.data(), xptr, xld, n, r);
      if (he != hipSuccess) {
        e = dcx_fail_hip(he, "copy of the solution to the host");
        break;
      }
      colmax(hd, dn);
      colmax(hx, xn);
      bool all_small = true, any_grow = false, left_small = it > 0;
      last = 0.0;
      for (int64_t c = 0; c < r; ++c) {
        if (!(dn[c] <= tol * xn[c])) all_small = false;
        if (it > 0 && dn[c] > 0.5 * prev[c]) any_grow = true;
        if (it > 0 && !(dcx_remaining_error(dn[c], prev[c]) <= tol * xn[c])) left_small = false;
        last = std::max(last, xn[c] > 0 ? dn[c] / xn[c] : dn[c]);
      }
      if (any_grow && !all_small) break;   // stagnation: d not added
      e = submit(rt, DC_AXPY, {hR, X}, {DC_R, DC_RW}, 0);
      if (!e) e = dc_wait_all(rt);
      if (e) break;
      if (all_small || left_small) { converged = true; break; }
      if (++it >= maxit) break;
      prev = dn;
    }
    if (inv && hV) dc_matrix_unpartition(rt, hV);
    dc_matrix_unpartition(rt, hW);
    TRY(e);
    rep->refine_ms = now_ms() - t1;
    rep->iterations = it;
    rep->converged = converged ? 1 : 0;
    rep->last_update = last;
    rep->final_prec = prec;
    if (converged || prec == DC_F64) return 0;
    prec = prec == DC_BF16 ? DC_F32 : DC_F64;
    rep->fallbacks++;
  }
}

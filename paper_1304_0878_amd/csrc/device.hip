// Device side of dagchol: the level executor and the tile kernels it runs.
//
// The host splits the task graph (the access-mode graph of the paper's
// Section 2) into levels: every task of a level has all its predecessors in
// earlier levels.  Each level is one launch of dc_level_kernel; its
// workgroups (256 threads, four 64-wide waves) take work units from the
// level's list through an atomic counter until the list is exhausted.  A
// task may be split into several units (sub-blocks of its output).  No
// workgroup ever waits for another: ordering between levels comes from the
// stream order of the launches.
//
// This file holds the panel kernel: every unit kind except the GEMM/SYRK
// updates, which run in their own kernel (gemm_kernel.hip) concurrently with
// it.  Tile kernels (right-looking tiled Cholesky; the paper's Section 5.1
// cites Cholesky as the partitioning idiom):
//   POTRF  D = L L^T on one diagonal tile (FP64, left-looking 16-column
//          panels: MFMA panel update, one wave factors the diagonal block,
//          the other rows follow by substitution).
//   TRSM   X <- X L^{-T} on 16-row slabs of a panel tile kept in LDS (FP64
//          arithmetic; FP32 tiles are widened on load and rounded on store,
//          optionally also writing a BF16 copy).
//   solve  forward/backward substitution and the RHS updates, FP64
//          arithmetic on FP64 or FP32 factor tiles.
//
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "exec_abi.h"
#include "queue_dev.h"

using namespace dcx;

namespace {

constexpr int NT = 256;                    // threads per workgroup
constexpr int LDS_DOUBLES = PANEL_LDS_DOUBLES;     // largest LDS need of a unit

static_assert(NT == 256 && PANEL == 16 && TRSM_ROWS == 16, "stage16 maps 256 threads on 16 rows");
static_assert(2 * TRSM_ROWS * (MAX_TILE + 2) + PANEL * (PANEL + 2) + PANEL <= LDS_DOUBLES, "trsm lds");
static_assert(PANEL * (MAX_TILE + 2) + PANEL * (PANEL + 2) + PANEL + 8 <= LDS_DOUBLES, "potrf lds");
static_assert(solve_lds_doubles(MAX_TILE) <= LDS_DOUBLES, "solve lds");

// Global-memory views of the tile pointers: descriptors hold generic
// pointers, and loads through them would otherwise be flat loads (which also
// count against the LDS wait counter and serialize with LDS traffic).
typedef __attribute__((address_space(1))) double gdouble;
typedef double dvec2 __attribute__((ext_vector_type(2)));
typedef __attribute__((address_space(1))) dvec2 gdvec2;
typedef __attribute__((address_space(1))) float gfloat;
typedef __attribute__((address_space(1))) __bf16 gbf16;
template <typename T> using gptr = __attribute__((address_space(1))) T *;

__device__ __forceinline__ double mfma44(double a, double b, double c) {
  return __builtin_amdgcn_mfma_f64_4x4x4f64(a, b, c, 0, 0, 0);
}

// Copies a block of 16 rows x ncols of a row-major global matrix into LDS
// (row stride dstride); rows at or beyond nvalid are zero.  Thread t takes
// row t/16 and columns t%16 + 16i, so each wave reads four 128-byte row
// segments per instruction, and keeps eight loads in flight before its LDS
// stores.  TS is the storage type of the source (double or float).
template <typename TS>
__device__ __forceinline__ void stage16(double *dst, int dstride, gptr<const TS> src, int64_t ld,
                                        int nvalid, int ncols) {
  const int r = threadIdx.x >> 4, c = threadIdx.x & 15;
  gptr<const TS> sp = src + (int64_t)(r < nvalid ? r : 0) * ld;
  const bool ok = r < nvalid;
  for (int cb = 0; cb < ncols; cb += 128) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int cc = cb + c + 16 * u;
      v[u] = (ok && cc < ncols) ? (double)sp[cc] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int cc = cb + c + 16 * u;
      if (cc < ncols) dst[r * dstride + cc] = v[u];
    }
  }
}

// Orders the LDS accesses of one wave (its LDS operations execute in issue
// order; this keeps the compiler from moving them across the point).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Value of v on lane `lane` (a constant), in every lane.
__device__ __forceinline__ double readlane_f64(double v, int lane) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffff), lane);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// ------------------------------------------------------------------ TRSM
//
// X (m x nb) <- X L^{-T}; unit = 16 consecutive rows of X held in LDS.
// For each 16-column block J: the rows c0..c0+15 of L left of the block are
// staged in LDS; (1) X_J -= X_{<J} L_{J,<J}^T with MFMA, wave w producing
// columns 4w..4w+3 for all 16 rows; (2) one thread per row solves the 16x16
// lower-triangular system with L_JJ (divisions by the diagonal).
//
// With TRTRI the same substitution inverts L: the 16 rows are rows
// 16u..16u+15 of the identity, so X becomes rows of L^{-T}, i.e. columns of
// W = L^{-1}, stored transposed into W's lower triangle.  Those rows are zero
// left of column 16u, so the blocks and the update terms left of it are
// skipped.  Each unit also records max |W| over its columns in W[0][1 + u],
// and unit 0, which reads all of L's lower triangle, max |L| in W[1][2]: the
// strictly upper part of W is otherwise unused and is never written by the
// transposed store.
constexpr int INV_SLOT_ROW_W = 0;   // W[0][1 + u]: max |W| of unit u's columns
constexpr int INV_SLOT_L = 1;       // W[1][2]: max |L| over the lower triangle

// Largest value over the workgroup (all threads return it).
__device__ __forceinline__ double block_max(double v, double *red) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v = fmax(v, __shfl_xor(v, o));
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  v = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
  __syncthreads();
  return v;
}

template <bool TRTRI>
__device__ __forceinline__ void trsm_core(const TaskDesc &d, int unit, double *lds,
                                          const gdouble *L, int64_t ldl) {
  const int nb = d.n;
  const int r0 = unit * TRSM_ROWS;
  const int rows = min(TRSM_ROWS, d.m - r0);
  const int XS = panel_stride(nb);
  gdouble *X = (gdouble *)d.c + (int64_t)r0 * d.ldc;
  const int64_t ldc = d.ldc;
  double *Xs = lds;                          // 16 x XS
  double *Lp = lds + TRSM_ROWS * XS;         // 16 x XS
  // diagonal block of the panel, transposed (l_pj in Ljt[j][p], stride 18:
  // column j read in aligned pairs), and its reciprocal pivots
  double *Ljt = Lp + TRSM_ROWS * XS;         // 16 x 18
  double *Rj = Ljt + PANEL * (PANEL + 2);    // 16
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int w = tid >> 6;
  const int l16 = lane & 15;
  const int blk = l16 >> 2;
  const int kq = lane >> 4;
  const int n4 = lane & 3;

  const bool x32 = !TRTRI && d.tc == T_F32;
  gfloat *X32 = (gfloat *)d.c + (int64_t)r0 * d.ldc;
  if (TRTRI) {
    for (int idx = tid; idx < TRSM_ROWS * nb; idx += NT) {
      const int r = idx / nb, c = idx - r * nb;
      Xs[r * XS + c] = (r < rows && c == r0 + r) ? 1.0 : 0.0;
    }
  } else if (x32) {
    stage16<float>(Xs, XS, X32, ldc, rows, nb);
  } else {
    stage16<double>(Xs, XS, X, ldc, rows, nb);
  }
  // identity rows are zero left of r0: neither blocks nor update terms
  // there contribute
  const int kstart = TRTRI ? r0 : 0;
  double lmax = 0.0;
  const int nj = (nb + PANEL - 1) / PANEL;
  for (int J = TRTRI ? unit : 0; J < nj; ++J) {
    const int c0 = PANEL * J;
    const int wj = min(PANEL, nb - c0);
    // rows c0..c0+15 of L, columns kstart..c0+15 (the block left of the
    // diagonal and the diagonal block itself)
    stage16<double>(Lp + kstart, XS, L + (int64_t)c0 * ldl + kstart, ldl, wj, c0 + wj - kstart);
    __syncthreads();
    {
      const int i = tid >> 4, j = tid & 15;
      const double lij = (i < wj && j <= i) ? Lp[i * XS + c0 + j] : 0.0;
      Ljt[j * (PANEL + 2) + i] = lij;
      if (i == j) Rj[i] = i < wj ? 1.0 / lij : 0.0;
    }
    if (TRTRI && unit == 0) {
      // lower-triangle entries of the staged rows
      for (int idx = tid; idx < PANEL * (c0 + PANEL); idx += NT) {
        const int i = idx / (c0 + PANEL), c = idx - i * (c0 + PANEL);
        if (i < wj && c <= c0 + i) lmax = fmax(lmax, fabs(Lp[i * XS + c]));
      }
    }
    __syncthreads();
    if (c0 > kstart) {
      double acc = 0.0;
      const double *xa = Xs + l16 * XS + kq;
      const double *lb = Lp + (4 * w + n4) * XS + kq;
      for (int k0 = kstart; k0 < c0; k0 += 16) {
#pragma unroll
        for (int j = 0; j < 4; ++j) acc = mfma44(xa[k0 + 4 * j], lb[k0 + 4 * j], acc);
      }
      const int row = 4 * blk + kq;
      const int col = 4 * w + n4;
      if (col < wj) Xs[row * XS + c0 + col] -= acc;
    }
    __syncthreads();
    if (tid < rows) {
      // right-looking substitution with the reciprocal pivots; column j + 1
      // of the block is read while column j is applied
      double v[PANEL];
      double *xr = Xs + tid * XS + c0;
#pragma unroll
      for (int j = 0; j < PANEL; ++j) v[j] = j < wj ? xr[j] : 0.0;
      double cur[PANEL], nxt[PANEL];
      cur[0] = Rj[0];
#pragma unroll
      for (int p = 1; p < PANEL; ++p) cur[p] = Ljt[p];
#pragma unroll
      for (int j = 0; j < PANEL; ++j) {
        if (j + 1 < PANEL) {
          nxt[0] = Rj[j + 1];
#pragma unroll
          for (int p = j + 2; p < PANEL; ++p) nxt[p] = Ljt[(j + 1) * (PANEL + 2) + p];
        }
        __builtin_amdgcn_sched_barrier(0);
        if (j < wj) {
          v[j] *= cur[0];
#pragma unroll
          for (int p = j + 1; p < PANEL; ++p) v[p] = fma(-v[j], cur[p], v[p]);
        }
        __builtin_amdgcn_sched_barrier(0);
        cur[0] = nxt[0];
#pragma unroll
        for (int p = j + 2; p < PANEL; ++p) cur[p] = nxt[p];
      }
#pragma unroll
      for (int j = 0; j < PANEL; ++j)
        if (j < wj) xr[j] = v[j];
    }
    __syncthreads();
  }
  if (TRTRI) {
    // W[c][r0 + r] = X[r][c] on and below the diagonal; 16 consecutive
    // threads write 16 consecutive entries of one row of W
    double wmax = 0.0;
    for (int idx = tid; idx < TRSM_ROWS * nb; idx += NT) {
      const int r = idx & 15, c = idx >> 4;
      if (r < rows && c >= r0 + r) {
        const double v = Xs[r * XS + c];
        wmax = fmax(wmax, fabs(v));
        ((gdouble *)d.c)[(int64_t)c * ldc + r0 + r] = v;
      }
    }
    wmax = block_max(wmax, Ljt);
    lmax = block_max(lmax, Ljt);
    if (tid == 0) {
      ((gdouble *)d.c)[(int64_t)INV_SLOT_ROW_W * ldc + 1 + unit] = wmax;
      if (unit == 0) ((gdouble *)d.c)[(int64_t)INV_SLOT_L * ldc + 2] = lmax;
    }
    return;
  }
  gbf16 *S16 = d.d ? (gbf16 *)d.d + (int64_t)r0 * d.ldd : nullptr;
  for (int idx = tid; idx < rows * nb; idx += NT) {
    const int r = idx / nb, c = idx - r * nb;
    if (x32) {
      const float v = (float)Xs[r * XS + c];
      X32[(int64_t)r * ldc + c] = v;
      if (S16) S16[(int64_t)r * d.ldd + c] = (__bf16)v;
    } else {
      X[(int64_t)r * ldc + c] = Xs[r * XS + c];
    }
  }
}

__device__ __forceinline__ void run_trsm(const TaskDesc &d, int unit, double *lds) {
  trsm_core<false>(d, unit, lds, (const gdouble *)d.a, d.lda);
}

// ------------------------------------------------------------- TRSM_INV
//
// X (m x nb) <- X W^T with W = L^{-1} from a TRTRI task: a dense product, so
// the substitution's column-by-column dependence disappears.  Unit = 16 rows
// of X staged in LDS; wave w produces the 16x16 output blocks b = w + 4i
// (interleaved so the triangular work is balanced over the waves) with
// 16x16x4 FP64 MFMA.  Block b only needs K chunks kc <= b (W is lower
// triangular); W's rows are streamed from global memory straight into the
// B operand, the next chunk's loads in flight while the current one is
// multiplied.  Inside a chunk, lane group kq takes the four consecutive k
// 4kq..4kq+3 (one 32-byte load per row) for the four MFMA steps, and the A
// operand follows the same order.
//
// The explicit inverse multiplies rounding errors by about max|L| max|W|;
// when the slots TRTRI recorded put that product above INV_LIMIT (or it is
// not finite) the unit solves with L by substitution instead, as a TRSM
// unit would, so ill-conditioned diagonal tiles keep the substitution's
// accuracy.
constexpr double INV_LIMIT = 1024.0;

template <bool FULL>
__device__ __forceinline__ void trsm_inv_product(const TaskDesc &d, int unit, double *lds) {
  const int nb = d.n;
  const int nb16 = (nb + 15) / 16;
  const int r0 = unit * TRSM_ROWS;
  const int rows = min(TRSM_ROWS, d.m - r0);
  const int XS = panel_stride(nb);
  const gdouble *W = (const gdouble *)d.a;
  const int64_t ldw = d.lda;
  const int64_t ldc = d.ldc;
  const bool x32 = d.tc == T_F32;
  double *Xs = lds;
  if (x32)
    stage16<float>(Xs, XS, (gfloat *)d.c + (int64_t)r0 * ldc, ldc, rows, nb);
  else
    stage16<double>(Xs, XS, (gdouble *)d.c + (int64_t)r0 * ldc, ldc, rows, nb);
  __syncthreads();
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int l16 = lane & 15, kq = lane >> 4;
  typedef double dvec4 __attribute__((ext_vector_type(4)));
  dvec4 acc[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) acc[i] = dvec4{0.0, 0.0, 0.0, 0.0};
  // B operand of block b, chunk kc: W[16b + l16][16kc + 4kq + s], s < 4
  auto wload = [&](int kc, double (&v)[8][4]) {
    const int k = 16 * kc + 4 * kq;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int b = w + 4 * i;
      if (b >= kc && b < nb16) {
        const int row = 16 * b + l16;
        if (FULL) {
          const gdvec2 *p = (const gdvec2 *)(W + (int64_t)row * ldw + k);
          const dvec2 x0 = p[0], x1 = p[1];
          v[i][0] = x0[0]; v[i][1] = x0[1]; v[i][2] = x1[0]; v[i][3] = x1[1];
        } else {
#pragma unroll
          for (int s = 0; s < 4; ++s)
            v[i][s] = (row < nb && k + s < nb) ? W[(int64_t)row * ldw + k + s] : 0.0;
        }
        if (b == kc) {   // diagonal chunk: only k <= row is part of W
#pragma unroll
          for (int s = 0; s < 4; ++s)
            if (4 * kq + s > l16) v[i][s] = 0.0;
        }
      }
    }
  };
  auto chunk = [&](int kc, const double (&v)[8][4]) {
    double a[4];
    const int k = 16 * kc + 4 * kq;
#pragma unroll
    for (int s = 0; s < 4; ++s) a[s] = (FULL || k + s < nb) ? Xs[l16 * XS + k + s] : 0.0;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int b = w + 4 * i;
      if (b >= kc && b < nb16) {
#pragma unroll
        for (int s = 0; s < 4; ++s)
          acc[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[s], v[i][s], acc[i], 0, 0, 0);
      }
    }
  };
  // two register sets alternate: the loads of one chunk are in flight while
  // the other is multiplied
  double wa[8][4], wb[8][4];
  wload(0, wa);
  for (int kc = 0; kc < nb16; kc += 2) {
    if (kc + 1 < nb16) wload(kc + 1, wb);
    chunk(kc, wa);
    if (kc + 2 < nb16) wload(kc + 2, wa);
    if (kc + 1 < nb16) chunk(kc + 1, wb);
  }
  // result element e of lane l: row l/16 + 4e, column l%16 of block b
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const int b = w + 4 * i;
    const int col = 16 * b + l16;
    if (b < nb16 && col < nb) {
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int row = kq + 4 * e;
        if (row < rows) {
          if (x32) {
            const float v = (float)acc[i][e];
            ((gfloat *)d.c)[(int64_t)(r0 + row) * ldc + col] = v;
            if (d.d) ((gbf16 *)d.d)[(int64_t)(r0 + row) * d.ldd + col] = (__bf16)v;
          } else {
            ((gdouble *)d.c)[(int64_t)(r0 + row) * ldc + col] = acc[i][e];
          }
        }
      }
    }
  }
}

// Diagonal step of a solve through W = L^{-1}, out of place: D <- W S
// (forward) or D <- W^T S (backward), S and D nb x r.  A unit is one 16-row
// block of D by 16 columns, so a step spreads over nb/16 x r/16 workgroups
// that stream disjoint rows (forward) or columns (backward) of W.  The 16
// columns of S are staged as the 16 rows of X = S^T over the K range the
// block needs (k <= i forward, k >= i backward); out[c][i] =
// sum_k X[c][k] Wop[i][k], Wop = W or W^T, with 16x16x4 FP64 MFMA.  The
// four waves take every fourth 16-column chunk of that range and their
// partial sums are added in LDS in wave order (a fixed order: the result
// does not depend on timing).
template <bool FULL, bool FWD>
__device__ __forceinline__ void solve_inv_product(const TaskDesc &d, int unit, double *lds) {
  const int nb = d.m, r = d.n;
  const int nb16 = (nb + 15) / 16;
  const int ncc = (r + 15) / 16;
  const int b = unit / ncc, c0 = 16 * (unit - b * ncc);   // b < nb16 by the unit count
  const int rc = min(16, r - c0);
  const int XS = panel_stride(nb);
  const gdouble *W = (const gdouble *)d.a;
  const int64_t ldw = d.lda;
  const gdouble *Sm = (const gdouble *)d.c;
  gdouble *Dm = (gdouble *)d.d;
  static_assert(SOLVE_INV_ROWS == 16, "one 16-row block per unit");
  const int kc_lo = FWD ? 0 : b;
  const int kc_hi = FWD ? b + 1 : nb16;   // exclusive
  const int k_lo = 16 * kc_lo, k_hi = min(nb, 16 * kc_hi);
  double *Xs = lds;                      // 16 x XS
  double *red = lds + 16 * XS;           // partial sums of waves 1..3
  for (int idx = threadIdx.x; idx < 16 * (k_hi - k_lo); idx += NT) {
    const int k = k_lo + (idx >> 4), c = idx & 15;
    Xs[c * XS + k] = c < rc ? Sm[(int64_t)k * d.ldc + c0 + c] : 0.0;
  }
  __syncthreads();
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int l16 = lane & 15, kq = lane >> 4;
  const int col = 16 * b + l16;          // output row i of this lane
  typedef double dvec4 __attribute__((ext_vector_type(4)));
  dvec4 acc = dvec4{0.0, 0.0, 0.0, 0.0};
  auto wload = [&](int kc, double (&v)[4]) {
    const int k = 16 * kc + 4 * kq;
    if (!FWD) {
#pragma unroll
      for (int s = 0; s < 4; ++s)
        v[s] = (FULL || (col < nb && k + s < nb)) ? W[(int64_t)(k + s) * ldw + col] : 0.0;
    } else if (FULL) {
      const gdvec2 *p = (const gdvec2 *)(W + (int64_t)col * ldw + k);
      const dvec2 x0 = p[0], x1 = p[1];
      v[0] = x0[0]; v[1] = x0[1]; v[2] = x1[0]; v[3] = x1[1];
    } else {
#pragma unroll
      for (int s = 0; s < 4; ++s)
        v[s] = (col < nb && k + s < nb) ? W[(int64_t)col * ldw + k + s] : 0.0;
    }
    if (kc == b) {   // diagonal chunk: only the triangle of W is read
#pragma unroll
      for (int s = 0; s < 4; ++s)
        if (FWD ? 4 * kq + s > l16 : 4 * kq + s < l16) v[s] = 0.0;
    }
  };
  auto chunk = [&](int kc, const double (&v)[4]) {
    const int k = 16 * kc + 4 * kq;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const double a = (FULL || k + s < nb) ? Xs[l16 * XS + k + s] : 0.0;
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, v[s], acc, 0, 0, 0);
    }
  };
  // wave w takes chunks kc_lo + w, + 4, + 8, ...; four of them in flight
  double v0[4] = {0, 0, 0, 0}, v1[4] = {0, 0, 0, 0}, v2[4] = {0, 0, 0, 0}, v3[4] = {0, 0, 0, 0};
  for (int kc = kc_lo + w; kc < kc_hi; kc += 16) {
    wload(kc, v0);
    if (kc + 4 < kc_hi) wload(kc + 4, v1);
    if (kc + 8 < kc_hi) wload(kc + 8, v2);
    if (kc + 12 < kc_hi) wload(kc + 12, v3);
    chunk(kc, v0);
    if (kc + 4 < kc_hi) chunk(kc + 4, v1);
    if (kc + 8 < kc_hi) chunk(kc + 8, v2);
    if (kc + 12 < kc_hi) chunk(kc + 12, v3);
  }
  if (w > 0) {
#pragma unroll
    for (int e = 0; e < 4; ++e) red[((w - 1) * 4 + e) * 64 + lane] = acc[e];
  }
  __syncthreads();
  // result element e of lane l: row (right-hand side) l/16 + 4e, column
  // (row i of D) l%16 of the block
  if (w == 0 && col < nb) {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      double v = acc[e];
      for (int q = 0; q < 3; ++q) v += red[(q * 4 + e) * 64 + lane];
      const int c = kq + 4 * e;
      if (c < rc) Dm[(int64_t)col * d.ldd + c0 + c] = v;
    }
  }
}

// Whether a task through W may use the inverse: max|L| * max|W| from the
// slots TRTRI wrote into W's strictly upper part.
__device__ __forceinline__ bool inverse_usable(const TaskDesc &d, int nb) {
  const int nb16 = (nb + 15) / 16;
  const gdouble *W = (const gdouble *)d.a;
  double wmax = 0.0;
  for (int u = 0; u < nb16; ++u) wmax = fmax(wmax, W[(int64_t)INV_SLOT_ROW_W * d.lda + 1 + u]);
  const double lmax = W[(int64_t)INV_SLOT_L * d.lda + 2];
  return __builtin_amdgcn_readfirstlane(wmax * lmax <= INV_LIMIT ? 1 : 0) != 0;
}

__device__ __forceinline__ bool inverse_full(const TaskDesc &d, int nb) {
  return nb % 16 == 0 && d.lda % 2 == 0 && ((uintptr_t)d.a & 15) == 0;
}

__device__ __forceinline__ void run_trsm_inv(const TaskDesc &d, int unit, double *lds) {
  if (!inverse_usable(d, d.n))
    trsm_core<false>(d, unit, lds, (const gdouble *)d.b, d.ldb);
  else if (inverse_full(d, d.n))
    trsm_inv_product<true>(d, unit, lds);
  else
    trsm_inv_product<false>(d, unit, lds);
}

// ----------------------------------------------------------------- POTRF
//
// Register-resident POTRF of a diagonal tile of order nb <= RPOTRF_MAX.  The
// lower triangle is cut into 16x16 blocks (I, J), J <= I, of MB block rows.
// Block column 0 goes from memory straight to LDS; the blocks with J >= 1
// live in MFMA accumulators (lane l holds rows 16I + l/16 + 4e, e = 0..3, of
// column 16J + l%16: the result layout of v_mfma_f64_16x16x4f64).  Wave w
// holds block rows w, 7 - w, 8 + w and 15 - w: the first two have 7 blocks
// with J >= 1 between them and the last two 23, for every w, so each wave
// has 30 slots, and slot s maps to its block with one comparison
// (rp_slot).
// Right-looking over the block columns k (the blocks of column k are in LDS
// when step k starts: column 0 from memory, column k + 1 published by the
// update of step k, which finishes it):
//  (1) the first wave factors the diagonal block in registers, lane i
//      holding row i (every row of 16 lanes holds the block): for each
//      column j the pivot is taken from lane j, its reciprocal square root r
//      is formed once (hardware estimate and two Newton steps) with
//      l_jj = pivot * r, column j is scaled by r, and the columns right of
//      it take a rank-one update whose column-j entries come from their
//      lanes by a DPP row broadcast; the block is stored, and published
//      with the reciprocals of its diagonal for step (2);
//  (2) every thread takes one row below the diagonal block and solves it by
//      substitution in the same column order (multiplying by the published
//      reciprocals), then stores and publishes it;
//  (3) each wave subtracts P_I P_J^T from its blocks right of column k with
//      four MFMAs (K = 16), RP_UGROUP slots at a time: a group with no block
//      right of column k is skipped, otherwise the operands of its slots are
//      read and their MFMA chains interleaved (a group may run a slot whose
//      block is finished or outside the tile: its accumulator is never read
//      again, and its operand rows are clamped into the buffer); the
//      group's blocks of column k + 1, now final, are published to the
//      other panel buffer for step k + 1.
// Rows and columns beyond nb are padded with the identity, which factors to
// itself and leaves the real entries unchanged.  Returns 0, or the 1-based
// column (within the tile) of the first non-positive or NaN pivot; the block
// columns left of that pivot's block hold their final values.
constexpr int RP_MB = RPOTRF_MAX / 16;
constexpr int RP_SLOTS = (RP_MB * (RP_MB - 1) / 2 + 3) / 4;   // 30
static_assert(RP_MB == 16 && RP_SLOTS == 30, "the row pairing of rp_slot assumes 16 block rows");
constexpr int RP_LD = PANEL + 1;                              // 17
constexpr int RP_LDT = PANEL + 2;                             // 18
constexpr int RP_GROUP = 6;                                   // slots loaded together
constexpr int RP_UGROUP = 4;                                  // slots updated together

typedef double dvec4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ dvec4 mfma16(double a, double b, dvec4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Block (I, J) of slot s of wave w (both wave-uniform, s a constant after
// unrolling): slots 0..6 run along rows w (J = 1..w) then 7 - w, slots 7..29
// along rows 8 + w then 15 - w.  The block exists in a tile of MB block rows
// when I < MB.
__device__ __forceinline__ void rp_slot(int s, int w, int &I, int &J) {
  if (s < 7) {
    const bool first = s < w;
    I = first ? w : 7 - w;
    J = first ? 1 + s : 1 + s - w;
  } else {
    const int t = s - 7;
    const bool first = t < 8 + w;
    I = first ? 8 + w : 15 - w;
    J = first ? 1 + t : 1 + t - 8 - w;
  }
}

// Value of v on lane p of each row of 16 lanes, in every lane of that row
// (DPP row_newbcast; p a constant after unrolling: the control is encoded in
// the instruction, hence the switch).
__device__ __forceinline__ double row_bcast(double v, int p) {
#define RB(q) case q: return __builtin_amdgcn_update_dpp(0.0, v, 0x150 + q, 0xf, 0xf, false)
  switch (p) {
    RB(0); RB(1); RB(2); RB(3); RB(4); RB(5); RB(6); RB(7);
    RB(8); RB(9); RB(10); RB(11); RB(12); RB(13); RB(14); default: RB(15);
  }
#undef RB
}

// 1 / sqrt(x) for a positive normal x: the hardware estimate refined by two
// Newton steps, r <- r + r (1 - x r^2) / 2 (quadratic convergence from the
// estimate's relative error, well below 2^-20, to rounding level; exact for
// powers of four).
__device__ __forceinline__ double rsqrt_nr(double x) {
  double r = __builtin_amdgcn_rsq(x);
#pragma unroll
  for (int it = 0; it < 2; ++it) {
    const double e = fma(-x * r, r, 1.0);
    r = fma(0.5 * r, e, r);
  }
  return r;
}

template <typename TS>
__device__ __forceinline__ int run_potrf_regs(const TaskDesc &d, double *lds) {
  const int nb = d.m;
  gptr<TS> D = (gptr<TS>)d.c;
  const int64_t ldd = d.ldc;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int l16 = lane & 15, kq = lane >> 4;
  const int MB = __builtin_amdgcn_readfirstlane((nb + 15) / 16);
  const int npad = 16 * MB;
  // two panel buffers of npad rows (step k uses buffer k % 2; addresses are
  // formed from lds so that they stay LDS addresses)
  const int pbuf = npad * RP_LD;
  // pivot block, transposed: l_pj in Lt[j][p] (zero above the diagonal),
  // with an even stride so that column j is read in aligned pairs; 1 / l_jj
  // in Rinv[j]
  double *Lt = lds + 2 * pbuf;
  double *Rinv = Lt + PANEL * RP_LDT;
  int *flag = (int *)(Rinv + PANEL);

  // block column 0 into the first panel buffer (identity padding): thread t
  // copies row t, its 16 loads (indices clamped in bounds) issued together
  if (tid < npad) {
    const int row = tid;
    const int64_t roff = (int64_t)min(row, nb - 1) * ldd;
    double v[PANEL];
#pragma unroll
    for (int c = 0; c < PANEL; ++c) v[c] = (double)D[roff + min(c, nb - 1)];
    // every load issued before the first use (left to itself the scheduler
    // puts each use, and a wait, right after its load)
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int c = 0; c < PANEL; ++c)
      lds[row * RP_LD + c] = row < nb && c < nb && c <= row ? v[c] : (row == c ? 1.0 : 0.0);
  }
  // the other blocks into the accumulators, RP_GROUP slots at a time: every
  // element read is in bounds (indices clamped), so a group's loads carry no
  // branches and issue back to back
  dvec4 acc[RP_SLOTS];
#pragma unroll
  for (int g = 0; g < RP_SLOTS; g += RP_GROUP) {
    bool any = false;
#pragma unroll
    for (int s = g; s < g + RP_GROUP && s < RP_SLOTS; ++s) {
      int I, J;
      rp_slot(s, w, I, J);
      any |= I < MB;
    }
    if (any) {
      double v[RP_GROUP][4];
#pragma unroll
      for (int s = g; s < g + RP_GROUP && s < RP_SLOTS; ++s) {
        int I, J;
        rp_slot(s, w, I, J);
        const int colc = min(16 * J + l16, nb - 1);
#pragma unroll
        for (int e = 0; e < 4; ++e)
          v[s - g][e] = (double)D[(int64_t)min(16 * I + kq + 4 * e, nb - 1) * ldd + colc];
      }
      // the group's loads all issued before the first use
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int s = g; s < g + RP_GROUP && s < RP_SLOTS; ++s) {
        int I, J;
        rp_slot(s, w, I, J);
        const bool valid = I < MB;
        const int col = 16 * J + l16;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int row = 16 * I + kq + 4 * e;
          acc[s][e] = valid && row < nb && col < nb && col <= row ? v[s - g][e]
                                                                  : (row == col ? 1.0 : 0.0);
        }
      }
    } else {
#pragma unroll
      for (int s = g; s < g + RP_GROUP && s < RP_SLOTS; ++s) acc[s] = (dvec4){0.0, 0.0, 0.0, 0.0};
    }
  }

  int bad = 0;
  for (int k = 0; k < MB; ++k) {
    double *Pk = lds + (k & 1) * pbuf;
    // block column k (block rows k .. MB - 1) is in Pk once every wave has
    // finished the previous step
    __syncthreads();
    // (1) the first wave factors the diagonal block; lane i holds row i
    // (lanes 16..63 repeat rows 0..15 and store nothing)
    if (w == 0) {
      const int i = l16;
      double v[PANEL];
#pragma unroll
      for (int j = 0; j < PANEL; ++j) v[j] = Pk[(16 * k + i) * RP_LD + j];
      double rinv = 0.0;
      int f = 0;
      // no early exit (it would keep the loop from unrolling): after a
      // failed pivot the rest is computed on garbage and not stored
#pragma unroll
      for (int j = 0; j < PANEL; ++j) {
        const double piv = readlane_f64(v[j], j);
        if (!(piv > 0.0) && f == 0) f = j + 1;   // non-positive or NaN: uniform
        const double rj = rsqrt_nr(piv);
        const double djj = piv * rj;
        v[j] = i == j ? djj : v[j] * rj;
        if (i == j) rinv = rj;
        // rank-one update of the columns right of j (entries above the
        // diagonal take garbage and are never read); l_pj comes from lane p
        // of the lane's row of 16, which holds the whole block
#pragma unroll
        for (int p = j + 1; p < PANEL; ++p) v[p] = fma(-v[j], row_bcast(v[j], p), v[p]);
      }
      if (!f && kq == 0) {
        const int row = 16 * k + i;
#pragma unroll
        for (int j = 0; j < PANEL; ++j) {
          const double x = j <= i ? v[j] : 0.0;
          Lt[j * RP_LDT + i] = x;
          if (j <= i && row < nb) D[(int64_t)row * ldd + 16 * k + j] = (TS)x;
        }
        Rinv[i] = rinv;
      }
      if (lane == 0) *flag = f;
    }
    __syncthreads();
    {
      const int f = *flag;
      if (f) {
        // a pivot inside the padding cannot fail (it is 1)
        bad = 16 * k + f;
        break;
      }
    }
    // (2) rows below the diagonal block, one per thread, by substitution
    // with the published factor
    {
      const int row = 16 * (k + 1) + tid;
      if (row < npad) {
        double x[PANEL];
#pragma unroll
        for (int j = 0; j < PANEL; ++j) x[j] = Pk[row * RP_LD + j];
        // column j of the pivot block and 1 / l_jj are read while column
        // j - 1 is applied (left to itself the scheduler waits for each
        // read right after issuing it)
        double cur[PANEL], nxt[PANEL];
        cur[0] = Rinv[0];
#pragma unroll
        for (int p = 1; p < PANEL; ++p) cur[p] = Lt[p];
#pragma unroll
        for (int j = 0; j < PANEL; ++j) {
          if (j + 1 < PANEL) {
            nxt[0] = Rinv[j + 1];
#pragma unroll
            for (int p = j + 2; p < PANEL; ++p) nxt[p] = Lt[(j + 1) * RP_LDT + p];
          }
          __builtin_amdgcn_sched_barrier(0);
          x[j] *= cur[0];
#pragma unroll
          for (int p = j + 1; p < PANEL; ++p) x[p] = fma(-x[j], cur[p], x[p]);
          __builtin_amdgcn_sched_barrier(0);
          cur[0] = nxt[0];
#pragma unroll
          for (int p = j + 2; p < PANEL; ++p) cur[p] = nxt[p];
        }
#pragma unroll
        for (int j = 0; j < PANEL; ++j) Pk[row * RP_LD + j] = x[j];
        if (row < nb) {
          gptr<TS> Dr = D + (int64_t)row * ldd + 16 * k;
          if (16 * k + PANEL <= nb) {
#pragma unroll
            for (int j = 0; j < PANEL; ++j) Dr[j] = (TS)x[j];
          } else {
            // the last block column is narrower than 16
            for (int j = 0; j < nb - 16 * k; ++j) Dr[j] = (TS)Pk[row * RP_LD + j];
          }
        }
      }
    }
    __syncthreads();
    // (3) trailing update of this wave's blocks right of column k
#pragma unroll
    for (int g = 0; g < RP_SLOTS; g += RP_UGROUP) {
      const int gl = min(g + RP_UGROUP, RP_SLOTS) - 1;
      bool any = false;
#pragma unroll
      for (int s = g; s <= gl; ++s) {
        int I, J;
        rp_slot(s, w, I, J);
        any |= I < MB && J > k;
      }
      if (any) {
        double a[RP_UGROUP][4], b[RP_UGROUP][4];
#pragma unroll
        for (int s = g; s <= gl; ++s) {
          int I, J;
          rp_slot(s, w, I, J);
          const int ra = (16 * min(I, MB - 1) + l16) * RP_LD + kq;
          const int rb = (16 * min(J, MB - 1) + l16) * RP_LD + kq;
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            a[s - g][q] = -Pk[ra + 4 * q];
            b[s - g][q] = Pk[rb + 4 * q];
          }
        }
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
          for (int s = g; s <= gl; ++s) acc[s] = mfma16(a[s - g][q], b[s - g][q], acc[s]);
        // blocks of column k + 1 are final: publish them for the next step
        double *Pn = lds + ((k + 1) & 1) * pbuf;
#pragma unroll
        for (int s = g; s <= gl; ++s) {
          int I, J;
          rp_slot(s, w, I, J);
          if (J == k + 1 && I < MB) {
#pragma unroll
            for (int e = 0; e < 4; ++e) Pn[(16 * I + kq + 4 * e) * RP_LD + l16] = acc[s][e];
          }
        }
      }
    }
  }
  __syncthreads();
  return bad;
}

// Left-looking POTRF (orders above RPOTRF_MAX, up to MAX_TILE; the full
// instance runs it next to the other panel units).
//
// D (nb x nb, lower) = L L^T in place.  Left-looking over 16-column panels:
// (1) D[c0:, c0:c0+16] -= D[c0:, :c0] D[c0:c0+16, :c0]^T with MFMA: the 16
// pivot rows are staged in LDS, each wave takes every fourth 16-row group
// and keeps up to eight groups' accumulators, the next 16 columns of its
// rows being loaded while the current ones are multiplied; (2) the first
// wave factors the 16x16 diagonal block column by column (square root of
// each pivot, or breakdown), exchanging pivot rows through LDS inside the
// wave, and publishes it; after one barrier every thread finishes the rows
// below the block by substitution.  Returns 0 or the 1-based local column of
// the first non-positive pivot.
// TS: the storage type of the tile (double, or float for an FP32 factor:
// every value is widened on load, the arithmetic is FP64, and each store
// rounds to FP32).
template <typename TS>
__device__ __forceinline__ int run_potrf(const TaskDesc &d, double *lds) {
  const int nb = d.m;
  gptr<TS> D = (gptr<TS>)d.c;
  const int64_t ldd = d.ldc;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int w = tid >> 6;
  const int l16 = lane & 15;
  const int blk = l16 >> 2;
  const int kq = lane >> 4;
  const int n4 = lane & 3;
  const int BS = panel_stride(nb);
  double *Bp = lds;                          // 16 x BS: pivot rows left of the panel
  double *Ds = Bp + PANEL * BS;              // 16 x 17: published pivot rows
  int *flag = (int *)(Ds + PANEL * (PANEL + 1));
  constexpr int RPT = MAX_TILE / NT;         // row slots per thread
  constexpr int GQ = MAX_TILE / PANEL / 4;   // row groups per wave

  const int nj = (nb + PANEL - 1) / PANEL;
  int bad = 0;
  for (int J = 0; J < nj && !bad; ++J) {
    const int c0 = PANEL * J;
    const int wj = min(PANEL, nb - c0);
    const int nrows = nb - c0;
    if (c0 > 0) {
      stage16<TS>(Bp, BS, D + (int64_t)c0 * ldd, ldd, wj, c0);
      __syncthreads();
      const int ngroups = (nrows + 15) / 16;
      double acc[GQ][4];
      TS an[GQ][4];   // read ahead in the storage type, widened where used
      gptr<const TS> ap[GQ];
      bool aok[GQ];
#pragma unroll
      for (int q = 0; q < GQ; ++q) {
        const int row = c0 + 16 * (w + 4 * q) + l16;
        aok[q] = row < nb;
        ap[q] = D + (int64_t)(aok[q] ? row : c0) * ldd + kq;
#pragma unroll
        for (int s = 0; s < 4; ++s) acc[q][s] = 0.0;
#pragma unroll
        for (int j = 0; j < 4; ++j) an[q][j] = aok[q] ? ap[q][4 * j] : (TS)0;
      }
      for (int k0 = 0; k0 < c0; k0 += 16) {
        double ac[GQ][4];
#pragma unroll
        for (int q = 0; q < GQ; ++q)
#pragma unroll
          for (int j = 0; j < 4; ++j) ac[q][j] = (double)an[q][j];
        if (k0 + 16 < c0) {
#pragma unroll
          for (int q = 0; q < GQ; ++q)
            if (w + 4 * q < ngroups) {
#pragma unroll
              for (int j = 0; j < 4; ++j) an[q][j] = aok[q] ? ap[q][k0 + 16 + 4 * j] : (TS)0;
            }
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          double b[4];
#pragma unroll
          for (int s = 0; s < 4; ++s) b[s] = Bp[(4 * ((blk + s) & 3) + n4) * BS + k0 + 4 * j + kq];
#pragma unroll
          for (int q = 0; q < GQ; ++q)
            if (w + 4 * q < ngroups) {
#pragma unroll
              for (int s = 0; s < 4; ++s) acc[q][s] = mfma44(ac[q][j], b[s], acc[q][s]);
            }
        }
      }
#pragma unroll
      for (int q = 0; q < GQ; ++q) {
        if (w + 4 * q < ngroups) {
          const int row = c0 + 16 * (w + 4 * q) + 4 * blk + kq;
#pragma unroll
          for (int s = 0; s < 4; ++s) {
            const int col = 4 * ((blk + s) & 3) + n4;
            if (row < nb && col < wj && c0 + col <= row) {
              gptr<TS> p = D + (int64_t)row * ldd + c0 + col;
              *p = (TS)((double)*p - acc[q][s]);
            }
          }
        }
      }
      __syncthreads();
    }
    // factor of the panel: (a) the first wave factors the 16x16 diagonal
    // block, lane j owning row c0 + j, column by column with the finished
    // pivot rows exchanged through LDS inside the wave (no workgroup
    // barrier); (b) after one barrier every thread finishes its rows below
    // the block by substitution with the published block.
    double v[RPT][PANEL];
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      const int row = c0 + tid + NT * q;
#pragma unroll
      for (int j = 0; j < PANEL; ++j)
        v[q][j] = (row < nb && j < wj && c0 + j <= row) ? (double)D[(int64_t)row * ldd + c0 + j] : 0.0;
    }
    if (w == 0) {
      int f = 0;
#pragma unroll
      for (int j = 0; j < PANEL; ++j) {
        if (j < wj) {
          if (lane == j) {
            double s = v[0][j];
#pragma unroll
            for (int p = 0; p < j; ++p) s = s - v[0][p] * v[0][p];
            const bool okp = s > 0.0;
            v[0][j] = okp ? sqrt(s) : s;
#pragma unroll
            for (int p = 0; p <= j; ++p) Ds[j * (PANEL + 1) + p] = v[0][p];
            Ds[j * (PANEL + 1) + PANEL] = okp ? 0.0 : 1.0;
          }
          wave_sync();
          if (Ds[j * (PANEL + 1) + PANEL] != 0.0) {   // same value in every lane
            f = j + 1;
            break;
          }
          if (lane > j && lane < wj) {
            double t = v[0][j];
#pragma unroll
            for (int p = 0; p < j; ++p) t = t - v[0][p] * Ds[j * (PANEL + 1) + p];
            v[0][j] = t / Ds[j * (PANEL + 1) + j];
          }
        }
      }
      if (lane == 0) *flag = f;
    }
    __syncthreads();
    bad = *flag ? c0 + *flag : 0;
    if (!bad) {
#pragma unroll
      for (int q = 0; q < RPT; ++q) {
        const int row = c0 + tid + NT * q;
        if (row >= c0 + PANEL && row < nb) {
#pragma unroll
          for (int j = 0; j < PANEL; ++j) {
            if (j < wj) {
              double t = v[q][j];
#pragma unroll
              for (int p = 0; p < j; ++p) t = t - v[q][p] * Ds[j * (PANEL + 1) + p];
              v[q][j] = t / Ds[j * (PANEL + 1) + j];
            }
          }
        }
      }
    }
    if (!bad) {
#pragma unroll
      for (int q = 0; q < RPT; ++q) {
        const int row = c0 + tid + NT * q;
#pragma unroll
        for (int j = 0; j < PANEL; ++j)
          if (row < nb && j < wj && c0 + j <= row) D[(int64_t)row * ldd + c0 + j] = (TS)v[q][j];
      }
    }
    __syncthreads();
  }
  return bad;
}

// Left-looking POTRF, the instance of its own (orders above RPOTRF_MAX, up
// to MAX_TILE, in graphs without GEMM or SYRK units).
//
// D (nb x nb, lower) = L L^T in place.  Left-looking over 16-column panels:
// (1) D[c0:, c0:c0+16] -= D[c0:, :c0] D[c0:c0+16, :c0]^T with MFMA: the 16
// pivot rows are staged in LDS, each wave takes every fourth 16-row group
// and keeps up to eight groups' accumulators, the next 16 columns of its
// rows being loaded while the current ones are multiplied; (2) the first
// wave factors the 16x16 diagonal block in registers as the register-
// resident factor does (reciprocal square roots of the pivots, DPP row
// broadcasts), and publishes it; after one barrier every thread finishes
// its rows below the block by substitution.  Returns 0 or the 1-based local
// column of the first non-positive or NaN pivot; the panels left of it hold
// their final values.
// TS: the storage type of the tile (double, or float for an FP32 factor:
// every value is widened on load, the arithmetic is FP64, and each store
// rounds to FP32).
template <typename TS>
__device__ __forceinline__ int run_potrf_ll(const TaskDesc &d, double *lds) {
  const int nb = d.m;
  gptr<TS> D = (gptr<TS>)d.c;
  const int64_t ldd = d.ldc;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int w = tid >> 6;
  const int l16 = lane & 15;
  const int blk = l16 >> 2;
  const int kq = lane >> 4;
  const int n4 = lane & 3;
  const int BS = panel_stride(nb);
  double *Bp = lds;                          // 16 x BS: pivot rows left of the panel
  // the factored diagonal block, transposed (l_pj in Lt[j][p], zero above
  // the diagonal), and 1 / l_jj in Rinv[j]
  double *Lt = Bp + PANEL * BS;
  double *Rinv = Lt + PANEL * RP_LDT;
  int *flag = (int *)(Rinv + PANEL);
  constexpr int RPT = MAX_TILE / NT;         // row slots per thread
  constexpr int GQ = MAX_TILE / PANEL / 4;   // row groups per wave

  const int nj = (nb + PANEL - 1) / PANEL;
  int bad = 0;
  for (int J = 0; J < nj && !bad; ++J) {
    const int c0 = PANEL * J;
    const int wj = min(PANEL, nb - c0);
    const int nrows = nb - c0;
    if (c0 > 0) {
      stage16<TS>(Bp, BS, D + (int64_t)c0 * ldd, ldd, wj, c0);
      __syncthreads();
      const int ngroups = (nrows + 15) / 16;
      double acc[GQ][4];
      TS an[GQ][4];   // read ahead in the storage type, widened where used
      gptr<const TS> ap[GQ];
      bool aok[GQ];
#pragma unroll
      for (int q = 0; q < GQ; ++q) {
        const int row = c0 + 16 * (w + 4 * q) + l16;
        aok[q] = row < nb;
        ap[q] = D + (int64_t)(aok[q] ? row : c0) * ldd + kq;
#pragma unroll
        for (int s = 0; s < 4; ++s) acc[q][s] = 0.0;
#pragma unroll
        for (int j = 0; j < 4; ++j) an[q][j] = aok[q] ? ap[q][4 * j] : (TS)0;
      }
      for (int k0 = 0; k0 < c0; k0 += 16) {
        double ac[GQ][4];
#pragma unroll
        for (int q = 0; q < GQ; ++q)
#pragma unroll
          for (int j = 0; j < 4; ++j) ac[q][j] = (double)an[q][j];
        if (k0 + 16 < c0) {
#pragma unroll
          for (int q = 0; q < GQ; ++q)
            if (w + 4 * q < ngroups) {
#pragma unroll
              for (int j = 0; j < 4; ++j) an[q][j] = aok[q] ? ap[q][k0 + 16 + 4 * j] : (TS)0;
            }
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          double b[4];
#pragma unroll
          for (int s = 0; s < 4; ++s) b[s] = Bp[(4 * ((blk + s) & 3) + n4) * BS + k0 + 4 * j + kq];
#pragma unroll
          for (int q = 0; q < GQ; ++q)
            if (w + 4 * q < ngroups) {
#pragma unroll
              for (int s = 0; s < 4; ++s) acc[q][s] = mfma44(ac[q][j], b[s], acc[q][s]);
            }
        }
      }
#pragma unroll
      for (int q = 0; q < GQ; ++q) {
        if (w + 4 * q < ngroups) {
          const int row = c0 + 16 * (w + 4 * q) + 4 * blk + kq;
#pragma unroll
          for (int s = 0; s < 4; ++s) {
            const int col = 4 * ((blk + s) & 3) + n4;
            if (row < nb && col < wj && c0 + col <= row) {
              gptr<TS> p = D + (int64_t)row * ldd + c0 + col;
              *p = (TS)((double)*p - acc[q][s]);
            }
          }
        }
      }
      __syncthreads();
    }
    // factor of the panel: (a) the first wave factors the 16x16 diagonal
    // block in registers, lane i holding row c0 + i (each row of 16 lanes
    // the whole block; rows and columns past the tile padded with the
    // identity): per column a reciprocal square root of the pivot and a
    // rank-one update of the columns right of it through DPP row
    // broadcasts; it stores the block and publishes it transposed with the
    // reciprocals of its diagonal; (b) after one barrier every thread
    // finishes its rows below the block by substitution, multiplying by the
    // published reciprocals.
    if (w == 0) {
      const int i = l16;
      double dv[PANEL];
      {
        const int64_t roff = (int64_t)(c0 + min(i, wj - 1)) * ldd + c0;
#pragma unroll
        for (int j = 0; j < PANEL; ++j) dv[j] = (double)D[roff + min(j, wj - 1)];
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int j = 0; j < PANEL; ++j)
          dv[j] = i < wj && j < wj && j <= i ? dv[j] : (i == j ? 1.0 : 0.0);
      }
      double rinv = 0.0;
      int f = 0;
#pragma unroll
      for (int j = 0; j < PANEL; ++j) {
        const double piv = readlane_f64(dv[j], j);
        if (!(piv > 0.0) && f == 0) f = j + 1;   // non-positive or NaN: uniform
        const double rj = rsqrt_nr(piv);
        const double djj = piv * rj;
        dv[j] = i == j ? djj : dv[j] * rj;
        if (i == j) rinv = rj;
#pragma unroll
        for (int p = j + 1; p < PANEL; ++p) dv[p] = fma(-dv[j], row_bcast(dv[j], p), dv[p]);
      }
      if (!f && kq == 0) {
#pragma unroll
        for (int j = 0; j < PANEL; ++j) {
          const double x = j <= i ? dv[j] : 0.0;
          Lt[j * RP_LDT + i] = x;
          if (j <= i && i < wj) D[(int64_t)(c0 + i) * ldd + c0 + j] = (TS)x;
        }
        Rinv[i] = rinv;
      }
      if (lane == 0) *flag = f;
    }
    // the rows below the block (loaded while the block is factored)
    double v[RPT][PANEL];
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      const int row = c0 + PANEL + tid + NT * q;
      const int64_t roff = (int64_t)min(row, nb - 1) * ldd + c0;
#pragma unroll
      for (int j = 0; j < PANEL; ++j) v[q][j] = (double)D[roff + min(j, wj - 1)];
    }
    __syncthreads();
    bad = *flag ? c0 + *flag : 0;
    if (!bad) {
      // column j of the block and 1 / l_jj are read while column j - 1 is
      // applied; the columns past the tile (their l_pj zero) leave the rows
      // unchanged
      double cur[PANEL], nxt[PANEL];
      cur[0] = Rinv[0];
#pragma unroll
      for (int p = 1; p < PANEL; ++p) cur[p] = Lt[p];
#pragma unroll
      for (int j = 0; j < PANEL; ++j) {
        if (j + 1 < PANEL) {
          nxt[0] = Rinv[j + 1];
#pragma unroll
          for (int p = j + 2; p < PANEL; ++p) nxt[p] = Lt[(j + 1) * RP_LDT + p];
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int q = 0; q < RPT; ++q) v[q][j] *= cur[0];
#pragma unroll
        for (int p = j + 1; p < PANEL; ++p)
#pragma unroll
          for (int q = 0; q < RPT; ++q) v[q][p] = fma(-v[q][j], cur[p], v[q][p]);
        __builtin_amdgcn_sched_barrier(0);
        cur[0] = nxt[0];
#pragma unroll
        for (int p = j + 2; p < PANEL; ++p) cur[p] = nxt[p];
      }
#pragma unroll
      for (int q = 0; q < RPT; ++q) {
        const int row = c0 + PANEL + tid + NT * q;
        if (row < nb) {
#pragma unroll
          for (int j = 0; j < PANEL; ++j)
            if (j < wj) D[(int64_t)row * ldd + c0 + j] = (TS)v[q][j];
        }
      }
    }
    __syncthreads();
  }
  return bad;
}

// ----------------------------------------------------------------- solve
//
// Forward and backward substitution on one diagonal tile, and the
// right-hand-side updates between tiles.  FP64 arithmetic; L may be stored
// in FP64 or FP32.  All sums are split over 16 thread slices and reduced in
// a fixed order, so results do not depend on scheduling.

// Loads columns c0 .. c0 + rc - 1 (rc <= CW) of the right-hand sides into
// LDS (row stride BSS), rows nb .. nb16 - 1 zero; eight loads in flight.
template <int CW>
__device__ __forceinline__ void solve_stage(double *Bs, const gdouble *Bm, int64_t ldb, int nb,
                                            int nb16, int c0, int rc) {
  const int tid = threadIdx.x;
  for (int base = 0; base < nb16 * CW; base += NT * 8) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int idx = base + tid + NT * u, i = idx / CW, c = idx % CW;
      v[u] = (i < nb && c < rc) ? Bm[(int64_t)i * ldb + c0 + c] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int idx = base + tid + NT * u, i = idx / CW, c = idx % CW;
      if (i < nb16) Bs[i * BSS + c] = v[u];
    }
  }
}

// Solves the 16-row block at row i0 (h rows) in the first wave, once the
// partial sums are in part[row][slice][col]: lane (row q, column group g)
// reduces its row's slices in a fixed order, then the block is solved one
// row at a time, x_i = t_i * (1 / l_ii) on lane i shared across its column
// group, the other rows dropping their terms in x_i.  FORWARD: rows top down,
// lrow[i] = l_qi; otherwise bottom up with lrow[i] = l_iq.
template <bool FORWARD>
__device__ __forceinline__ void solve_block(double *Bs, const double *part, const double *Ljj,
                                            int i0, int h, int rc) {
  const int tid = threadIdx.x;
  if (tid >= 64) return;
  const int q = tid & 15, g = tid >> 4;
  double lrow[16];
#pragma unroll
  for (int p = 0; p < 16; ++p) lrow[p] = FORWARD ? Ljj[q * 17 + p] : Ljj[p * 17 + q];
  const double rinv = q < h ? 1.0 / Ljj[q * 17 + q] : 0.0;
  for (int cb = 0; cb < rc; cb += 4) {
    const int c = cb + g;
    double t = 0.0;
    if (q < h && c < rc) {
      double sum = 0.0;
#pragma unroll
      for (int sq = 0; sq < 16; ++sq) sum += part[(q * 16 + sq) * 16 + c];
      t = Bs[(i0 + q) * BSS + c] - sum;
    }
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      const int i = FORWARD ? k : 15 - k;
      if (i < h) {
        if (q == i) t = t * rinv;
        // x_i of each column group: lanes i, 16 + i, 32 + i, 48 + i
        double xi = readlane_f64(t, i);
        if (rc > 1) {
          const double x1 = readlane_f64(t, 16 + i), x2 = readlane_f64(t, 32 + i),
                       x3 = readlane_f64(t, 48 + i);
          xi = g == 1 ? x1 : g == 2 ? x2 : g == 3 ? x3 : xi;
        }
        if (FORWARD ? q > i : q < i) t = t - lrow[i] * xi;
      }
    }
    if (q < h && c < rc) Bs[(i0 + q) * BSS + c] = t;
  }
}

// B (nb x r) <- L^{-1} B (L lower); passes of up to CW columns in LDS.  Per
// 16-row block: (a) thread (row, slice) sums every 16th earlier term of its
// row, the row's loads all issued at once, and the block's diagonal part of
// L goes to LDS; (b, c) the first wave reduces and substitutes.
template <typename TL, int CW>
__device__ __forceinline__ void trsm_l_pass(const TaskDesc &d, double *lds, int c0, int rc) {
  const gptr<const TL> L = (const gptr<const TL>)d.a;
  const int64_t ldl = d.lda;
  gdouble *Bm = (gdouble *)d.c;
  const int64_t ldb = d.ldc;
  const int nb = d.m;
  const int tid = threadIdx.x;
  const int nb16 = (nb + 15) / 16 * 16;
  double *Bs = lds;                                // [nb16][BSS]
  double *part = Bs + nb16 * BSS;                  // [16][16][16]
  double *Ljj = part + 16 * 16 * 16 + 16 * 16;     // [16][17]
  const int ri = tid >> 4, sl = tid & 15;
  solve_stage<CW>(Bs, Bm, ldb, nb, nb16, c0, rc);
  // this thread's entries of L for a block at row i0: row i0 + ri, columns
  // sl + 16 u left of the block and the diagonal one; those of the next
  // block are loaded while the current block is being solved (kept in the
  // storage type and widened where used: a conversion next to each load
  // would make it wait for the load there)
  TL lv[MAX_TILE / 16];
  TL ldg = 0;
  auto lload = [&](int i0) {
    const int h = min(16, nb - i0), nu = i0 / 16;
    gptr<const TL> lr = L + (int64_t)(i0 + ri) * ldl;
#pragma unroll
    for (int u = 0; u < MAX_TILE / 16; ++u)
      lv[u] = (ri < h && u < nu) ? lr[sl + 16 * u] : (TL)0;
    ldg = (ri < h && sl <= ri) ? lr[i0 + sl] : (TL)0;
  };
  lload(0);
  __syncthreads();
  for (int i0 = 0; i0 < nb; i0 += 16) {
    const int h = min(16, nb - i0);
    const int nu = i0 / 16;   // earlier terms per slice (uniform)
    double acc[CW];
#pragma unroll
    for (int c = 0; c < CW; ++c) acc[c] = 0.0;
    if (ri < h) {
#pragma unroll
      for (int u = 0; u < MAX_TILE / 16; ++u) {
        if (u < nu) {
#pragma unroll
          for (int c = 0; c < CW; ++c) acc[c] += (double)lv[u] * Bs[(sl + 16 * u) * BSS + c];
        }
      }
      Ljj[ri * 17 + sl] = (double)ldg;
    }
#pragma unroll
    for (int c = 0; c < CW; ++c) part[(ri * 16 + sl) * 16 + c] = acc[c];
    if (i0 + 16 < nb) lload(i0 + 16);
    __syncthreads();
    solve_block<true>(Bs, part, Ljj, i0, h, rc);
    __syncthreads();
  }
  // in place, or into d.d (the out-of-place diagonal steps' fallback)
  gdouble *Bo = d.d ? (gdouble *)d.d : Bm;
  const int64_t ldo = d.d ? d.ldd : ldb;
  for (int idx = tid; idx < nb * CW; idx += NT) {
    const int i = idx / CW, c = idx % CW;
    if (c < rc) Bo[(int64_t)i * ldo + c0 + c] = Bs[i * BSS + c];
  }
  __syncthreads();
}

template <typename TL>
__device__ __forceinline__ void run_trsm_l(const TaskDesc &d, double *lds) {
  for (int c0 = 0; c0 < d.n; c0 += 16) {
    const int rc = min(16, d.n - c0);
    if (rc == 1) trsm_l_pass<TL, 1>(d, lds, c0, rc);
    else if (rc <= 4) trsm_l_pass<TL, 4>(d, lds, c0, rc);
    else trsm_l_pass<TL, 16>(d, lds, c0, rc);
  }
}

// B (nb x r) <- L^{-T} B: blocks from the bottom; the contribution of later
// rows p to row i uses L[p][i] (16 lanes read 16 consecutive entries of a
// row of L).
template <typename TL, int CW>
__device__ __forceinline__ void trsm_lt_pass(const TaskDesc &d, double *lds, int c0, int rc) {
  const gptr<const TL> L = (const gptr<const TL>)d.a;
  const int64_t ldl = d.lda;
  gdouble *Bm = (gdouble *)d.c;
  const int64_t ldb = d.ldc;
  const int nb = d.m;
  const int tid = threadIdx.x;
  const int nb16 = (nb + 15) / 16 * 16;
  double *Bs = lds;
  double *part = Bs + nb16 * BSS;
  double *Ljj = part + 16 * 16 * 16 + 16 * 16;
  const int ci = tid & 15, sl = tid >> 4;
  const int nblk = (nb + 15) / 16;
  solve_stage<CW>(Bs, Bm, ldb, nb, nb16, c0, rc);
  // this thread's entries of L for the block at row i0: column i0 + ci of
  // the later rows p = i0 + 16 + sl + 16 u (u < nu, uniform; rows past nb
  // read as zero and meet zero rows of Bs) and of the diagonal block; those
  // of the next block up are loaded while the current one is being solved
  // (in the storage type, widened where used)
  TL lv[MAX_TILE / 16];
  TL ldg = 0;
  auto lload = [&](int i0) {
    const int h = min(16, nb - i0), nu = (nb16 - i0 - 16) / 16;
#pragma unroll
    for (int u = 0; u < MAX_TILE / 16; ++u) {
      const int p = i0 + 16 + sl + 16 * u;
      lv[u] = (ci < h && u < nu && p < nb) ? L[(int64_t)p * ldl + i0 + ci] : (TL)0;
    }
    ldg = (sl < h && ci <= sl) ? L[(int64_t)(i0 + sl) * ldl + i0 + ci] : (TL)0;
  };
  lload(16 * (nblk - 1));
  __syncthreads();
  for (int bi = nblk - 1; bi >= 0; --bi) {
    const int i0 = 16 * bi;
    const int h = min(16, nb - i0);
    const int nu = (nb16 - i0 - 16) / 16;
    double acc[CW];
#pragma unroll
    for (int c = 0; c < CW; ++c) acc[c] = 0.0;
    if (ci < h) {
#pragma unroll
      for (int u = 0; u < MAX_TILE / 16; ++u) {
        if (u < nu) {
#pragma unroll
          for (int c = 0; c < CW; ++c) acc[c] += (double)lv[u] * Bs[(i0 + 16 + sl + 16 * u) * BSS + c];
        }
      }
    }
    // diagonal block, row sl of it: L[i0 + sl][i0 + ci]
    Ljj[sl * 17 + ci] = (double)ldg;
#pragma unroll
    for (int c = 0; c < CW; ++c) part[(ci * 16 + sl) * 16 + c] = acc[c];
    if (bi > 0) lload(i0 - 16);
    __syncthreads();
    solve_block<false>(Bs, part, Ljj, i0, h, rc);
    __syncthreads();
  }
  // in place, or into d.d (the out-of-place diagonal steps' fallback)
  gdouble *Bo = d.d ? (gdouble *)d.d : Bm;
  const int64_t ldo = d.d ? d.ldd : ldb;
  for (int idx = tid; idx < nb * CW; idx += NT) {
    const int i = idx / CW, c = idx % CW;
    if (c < rc) Bo[(int64_t)i * ldo + c0 + c] = Bs[i * BSS + c];
  }
  __syncthreads();
}

template <typename TL>
__device__ __forceinline__ void run_trsm_lt(const TaskDesc &d, double *lds) {
  for (int c0 = 0; c0 < d.n; c0 += 16) {
    const int rc = min(16, d.n - c0);
    if (rc == 1) trsm_lt_pass<TL, 1>(d, lds, c0, rc);
    else if (rc <= 4) trsm_lt_pass<TL, 4>(d, lds, c0, rc);
    else trsm_lt_pass<TL, 16>(d, lds, c0, rc);
  }
}

// Diagonal step of a solve through W = L^{-1} (TRSM_L_INV, TRSM_LT_INV),
// D <- L^{-1} S or L^{-T} S.  With an ill-conditioned L (see TRSM_INV) unit 0
// solves all columns by substitution with L, reading S and writing D, and
// the other units do nothing.
template <bool FWD>
__device__ __forceinline__ void run_trsm_l_inv(const TaskDesc &d, int unit, double *lds) {
  if (!inverse_usable(d, d.m)) {
    if (unit == 0) {
      TaskDesc dd = d;
      dd.a = d.b;
      dd.lda = d.ldb;
      dd.ta = T_F64;
      if (FWD) run_trsm_l<double>(dd, lds); else run_trsm_lt<double>(dd, lds);
    }
    return;
  }
  if (inverse_full(d, d.m))
    solve_inv_product<true, FWD>(d, unit, lds);
  else
    solve_inv_product<false, FWD>(d, unit, lds);
}

// B_I (m x r) -= L_IK (m x kb) Y_K (kb x r); unit = 16 rows, thread (row,
// slice) sums every 16th term with eight loads in flight; fixed-order
// reduction over the slices in LDS.
template <typename TL>
__device__ __forceinline__ void run_gemm_rhs_n(const TaskDesc &d, int unit, double *lds) {
  const gptr<const TL> L = (const gptr<const TL>)d.a;
  const gdouble *Y = (const gdouble *)d.b;
  gdouble *Bm = (gdouble *)d.c;
  const int m = d.m, r = d.n, kb = d.k;
  const int tid = threadIdx.x;
  const int ri = tid >> 4, sl = tid & 15;
  const int i0 = unit * RHS_ROWS;
  const int i = i0 + ri;
  double *part = lds;   // [16 rows][16 slices][8 cols]
  for (int c0 = 0; c0 < r; c0 += 8) {
    double acc[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) acc[c] = 0.0;
    if (i < m) {
      gptr<const TL> lr = L + (int64_t)i * d.lda;
      for (int pb = 0; pb < kb; pb += 128) {
        double lv[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int p = pb + sl + 16 * u;
          lv[u] = p < kb ? (double)lr[p] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int p = pb + sl + 16 * u;
          if (p < kb) {
            const gdouble *yp = Y + (int64_t)p * d.ldb + c0;
#pragma unroll
            for (int c = 0; c < 8; ++c)
              if (c0 + c < r) acc[c] += lv[u] * yp[c];
          }
        }
      }
    }
#pragma unroll
    for (int c = 0; c < 8; ++c) part[(ri * 16 + sl) * 8 + c] = acc[c];
    __syncthreads();
    if (sl < 8 && i < m && c0 + sl < r) {
      double sum = 0.0;
#pragma unroll
      for (int q = 0; q < 16; ++q) sum += part[(ri * 16 + q) * 8 + sl];
      gdouble *bp = Bm + (int64_t)i * d.ldc + c0 + sl;
      *bp = *bp - sum;
    }
    __syncthreads();
  }
}

// B_I (m x r) -= L_KI^T Y_K with L_KI (kb x m); unit = 16 output rows,
// thread (row, slice) reads L_KI[p][i] (16 consecutive entries of row p per
// 16 lanes); fixed-order reduction over the slices.
template <typename TL>
__device__ __forceinline__ void run_gemm_rhs_t(const TaskDesc &d, int unit, double *lds) {
  const gptr<const TL> L = (const gptr<const TL>)d.a;
  const gdouble *Y = (const gdouble *)d.b;
  gdouble *Bm = (gdouble *)d.c;
  const int m = d.m, r = d.n, kb = d.k;
  const int tid = threadIdx.x;
  const int ci = tid & 15, sl = tid >> 4;
  const int i0 = unit * RHS_ROWS;
  const int i = i0 + ci;
  double *part = lds;   // [16 rows][16 slices][8 cols]
  for (int c0 = 0; c0 < r; c0 += 8) {
    double acc[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) acc[c] = 0.0;
    if (i < m) {
      for (int pb = 0; pb < kb; pb += 128) {
        double lv[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int p = pb + sl + 16 * u;
          lv[u] = p < kb ? (double)L[(int64_t)p * d.lda + i] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int p = pb + sl + 16 * u;
          if (p < kb) {
            const gdouble *yp = Y + (int64_t)p * d.ldb + c0;
#pragma unroll
            for (int c = 0; c < 8; ++c)
              if (c0 + c < r) acc[c] += lv[u] * yp[c];
          }
        }
      }
    }
#pragma unroll
    for (int c = 0; c < 8; ++c) part[(ci * 16 + sl) * 8 + c] = acc[c];
    __syncthreads();
    {
      const int ro = tid >> 4, c = tid & 15;   // output row ro, column c
      const int io = i0 + ro;
      if (c < 8 && io < m && c0 + c < r) {
        double sum = 0.0;
#pragma unroll
        for (int q = 0; q < 16; ++q) sum += part[(ro * 16 + q) * 8 + c];
        gdouble *bp = Bm + (int64_t)io * d.ldc + c0 + c;
        *bp = *bp - sum;
      }
    }
    __syncthreads();
  }
}

// ------------------------------------------------------ elementwise tasks

// The paper's scale_vector task: x[i] *= factor (binary32).
__device__ __forceinline__ void run_scal(const TaskDesc &d, int unit) {
  gfloat *x = (gfloat *)d.c;
  const float f = (float)d.alpha;
  const int64_t base = (int64_t)unit * 4096;
  for (int64_t i = base + threadIdx.x; i < base + 4096 && i < d.m; i += NT) x[i] = x[i] * f;
}

__device__ __forceinline__ double load_as_f64(const void *p, int t, int64_t i) {
  if (t == T_F64) return ((const double *)p)[i];
  if (t == T_F32) return (double)((const float *)p)[i];
  return (double)(float)((const __bf16 *)p)[i];
}
__device__ __forceinline__ void store_from_f64(void *p, int t, int64_t i, double v) {
  if (t == T_F64) ((double *)p)[i] = v;
  else if (t == T_F32) ((float *)p)[i] = (float)v;
  else ((__bf16 *)p)[i] = (__bf16)(float)v;
}

// D (m x n) <- convert(S); unit = 64 rows.
__device__ __forceinline__ void run_cast(const TaskDesc &d, int unit) {
  const int r0 = unit * ROW_UNIT;
  const int rows = min(ROW_UNIT, d.m - r0);
  for (int64_t idx = threadIdx.x; idx < (int64_t)rows * d.n; idx += NT) {
    const int64_t r = r0 + idx / d.n, c = idx % d.n;
    const double v = load_as_f64(d.a, d.ta, r * d.lda + c);
    if (d.ta == T_F64 && d.tc == T_BF16)
      store_from_f64(d.c, d.tc, r * d.ldc + c, (double)(float)v);
    else
      store_from_f64(d.c, d.tc, r * d.ldc + c, v);
  }
}

// X (m x n) += D; unit = 64 rows.
__device__ __forceinline__ void run_axpy(const TaskDesc &d, int unit) {
  const int r0 = unit * ROW_UNIT;
  const int rows = min(ROW_UNIT, d.m - r0);
  const gdouble *D = (const gdouble *)d.a;
  gdouble *X = (gdouble *)d.c;
  for (int64_t idx = threadIdx.x; idx < (int64_t)rows * d.n; idx += NT) {
    const int64_t r = r0 + idx / d.n, c = idx % d.n;
    X[r * d.ldc + c] = X[r * d.ldc + c] + D[r * d.lda + c];
  }
}

// R (n x r) = B - A X, A symmetric (lower triangle read), FP64; unit = 64
// rows.  Part 1 (columns j <= i) reads rows of A, part 2 (j > i) reads the
// rows below the unit; each wave sums a slice and the slices are added in a
// fixed order.
// Error-free transformations (Ogita, Rump and Oishi, "Accurate sum and dot
// product", 2005): a*b = p + e exactly (one FMA), and a + b = s + t exactly.
__device__ __forceinline__ void two_prod(double a, double b, double &p, double &e) {
  p = a * b;
  e = __builtin_fma(a, b, -p);
}
__device__ __forceinline__ void two_sum(double a, double b, double &s, double &t) {
#pragma clang fp contract(off)
  s = a + b;
  const double z = s - a;
  t = (a - (s - z)) + (b - z);
}
// (s, c) += (s2, c2): compensated sum of two partial sums.
__device__ __forceinline__ void add2(double &s, double &c, double s2, double c2) {
#pragma clang fp contract(off)
  double t;
  two_sum(s, s2, s, t);
  c = c + (c2 + t);
}

// R <- B - A X with A symmetric (lower triangle stored); unit = 64 rows.
// Each row is a compensated dot product (Dot2 of the reference above: the
// products and sums are carried with their exact rounding errors), so the
// residual is as accurate as if computed in twice the FP64 precision and
// then rounded; iterative refinement then converges to a solution accurate
// to FP64 roundoff rather than to cond(A) times it.  Part 1: each wave takes
// 16 rows, lanes split the stored row (j <= i); part 2: lane = row, waves
// split the column below the diagonal (j > i), read coalesced.
constexpr int RB = 4;   // residual terms per lane in flight

__device__ __forceinline__ void run_resid(const TaskDesc &d, int unit, double *lds) {
#pragma clang fp contract(off)
  const gdouble *A = (const gdouble *)d.a;
  const gdouble *X = (const gdouble *)d.b;
  const gdouble *Bm = (const gdouble *)d.d;
  gdouble *R = (gdouble *)d.c;
  const int n = d.m, r = d.n;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int i0 = unit * ROW_UNIT;
  // [64 rows][4 cols] sums and errors of part 1, [4 slices][64][4] of part 2
  double *ps = lds, *pc = lds + 64 * 4;
  double *qs = lds + 2 * 64 * 4, *qc = qs + 4 * 64 * 4;
  for (int c0 = 0; c0 < r; c0 += 4) {
    for (int q = 0; q < 16; ++q) {
      const int ii = w * 16 + q;
      const int i = i0 + ii;
      double s[4], c[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) s[k] = c[k] = 0.0;
      if (i < n) {
        // RB terms per lane loaded before they are accumulated (same order
        // of accumulation, more loads in flight)
        const gdouble *ar = A + (int64_t)i * d.lda;
        for (int jb = lane; jb <= i; jb += RB * 64) {
          double av[RB], xv[RB][4];
#pragma unroll
          for (int u = 0; u < RB; ++u) {
            const int j = jb + 64 * u;
            av[u] = j <= i ? ar[j] : 0.0;
#pragma unroll
            for (int k = 0; k < 4; ++k)
              xv[u][k] = (j <= i && c0 + k < r) ? X[(int64_t)j * d.ldb + c0 + k] : 0.0;
          }
#pragma unroll
          for (int u = 0; u < RB; ++u) {
            if (jb + 64 * u <= i) {
#pragma unroll
              for (int k = 0; k < 4; ++k)
                if (c0 + k < r) {
                  double p, e, t;
                  two_prod(av[u], xv[u][k], p, e);
                  two_sum(s[k], p, s[k], t);
                  c[k] = c[k] + (t + e);
                }
            }
          }
        }
      }
#pragma unroll
      for (int k = 0; k < 4; ++k) {
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
          const double s2 = __shfl_xor(s[k], off), c2 = __shfl_xor(c[k], off);
          add2(s[k], c[k], s2, c2);
        }
        if (lane == 0) {
          ps[ii * 4 + k] = s[k];
          pc[ii * 4 + k] = c[k];
        }
      }
    }
    {
      const int ii = lane;
      const int i = i0 + ii;
      double s[4], c[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) s[k] = c[k] = 0.0;
      if (i < n) {
        for (int jb = i0 + 1 + w; jb < n; jb += RB * 4) {
          double av[RB], xv[RB][4];
#pragma unroll
          for (int u = 0; u < RB; ++u) {
            const int j = jb + 4 * u;
            const bool ok = j < n && j > i;
            av[u] = ok ? A[(int64_t)j * d.lda + i] : 0.0;
#pragma unroll
            for (int k = 0; k < 4; ++k)
              xv[u][k] = (ok && c0 + k < r) ? X[(int64_t)j * d.ldb + c0 + k] : 0.0;
          }
#pragma unroll
          for (int u = 0; u < RB; ++u) {
            const int j = jb + 4 * u;
            if (j < n && j > i) {
#pragma unroll
              for (int k = 0; k < 4; ++k)
                if (c0 + k < r) {
                  double p, e, t;
                  two_prod(av[u], xv[u][k], p, e);
                  two_sum(s[k], p, s[k], t);
                  c[k] = c[k] + (t + e);
                }
            }
          }
        }
      }
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        qs[(w * 64 + ii) * 4 + k] = s[k];
        qc[(w * 64 + ii) * 4 + k] = c[k];
      }
    }
    __syncthreads();
    if (tid < 64) {
      const int i = i0 + tid;
      if (i < n) {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          if (c0 + k < r) {
            double s = ps[tid * 4 + k], c = pc[tid * 4 + k];
#pragma unroll
            for (int sl = 0; sl < 4; ++sl)
              add2(s, c, qs[(sl * 64 + tid) * 4 + k], qc[(sl * 64 + tid) * 4 + k]);
            // r = b - (s + c), with the rounding of b - s kept
            double h, t;
            two_sum(Bm[(int64_t)i * d.ldd + c0 + k], -s, h, t);
            R[(int64_t)i * d.ldc + c0 + k] = h + (t - c);
          }
        }
      }
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------ level kernel

__device__ __forceinline__ uint64_t uniform_u64(uint64_t v) {
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
  return ((uint64_t)hi << 32) | lo;
}

// The units of the panel kernel, per instance.  Three instances, each
// compiled with only the units it runs so that its register allocation is
// its own: LI_FULL runs every kind (the factorisation's and the solves'
// units need up to about 500 registers per lane, so one workgroup per CU),
// LI_LIGHT the residual and elementwise units (RESID, CAST, AXPY, SCAL) and
// LI_RHS the right-hand-side updates of the solves (both keep to 128
// registers, four workgroups per CU: their units stream from memory).
template <int MODE>
__device__ __forceinline__ void run_panel_unit(const TaskDesc &d, int u, double *lds,
                                               int64_t *info, int32_t *failed) {
  const int kind = __builtin_amdgcn_readfirstlane(d.kind);
  if (MODE == LI_FULL || MODE == LI_LIGHT) switch (kind) {
    case K_SCAL: run_scal(d, u); break;
    case K_CAST: run_cast(d, u); break;
    case K_RESID: run_resid(d, u, lds); break;
    case K_AXPY: run_axpy(d, u); break;
    default: break;
  }
  if (MODE == LI_FULL || MODE == LI_RHS) switch (kind) {
    case K_GEMM_RHS_N:
      if (d.ta == T_F32) run_gemm_rhs_n<float>(d, u, lds); else run_gemm_rhs_n<double>(d, u, lds);
      break;
    case K_GEMM_RHS_T:
      if (d.ta == T_F32) run_gemm_rhs_t<float>(d, u, lds); else run_gemm_rhs_t<double>(d, u, lds);
      break;
    default: break;
  }
  if (MODE == LI_FULL) switch (kind) {
    case K_TRSM_L:
      if (d.ta == T_F32) run_trsm_l<float>(d, lds); else run_trsm_l<double>(d, lds);
      break;
    case K_TRSM_LT:
      if (d.ta == T_F32) run_trsm_lt<float>(d, lds); else run_trsm_lt<double>(d, lds);
      break;
    case K_TRSM_L_INV: run_trsm_l_inv<true>(d, u, lds); break;
    case K_TRSM_LT_INV: run_trsm_l_inv<false>(d, u, lds); break;
    case K_TRSM: case K_TRSM_CAST: run_trsm(d, u, lds); break;
    case K_TRTRI: trsm_core<true>(d, u, lds, (const gdouble *)d.a, d.lda); break;
    case K_TRSM_INV: case K_TRSM_INV_CAST: run_trsm_inv(d, u, lds); break;
    case K_POTRF: {
      const int bad = d.tc == T_F32 ? run_potrf<float>(d, lds) : run_potrf<double>(d, lds);
      if (bad && threadIdx.x == 0 && d.matrix >= 0) {
        info[d.matrix] = d.row0 + bad;
        failed[d.matrix] = 1;
      }
      break;
    }
    default: break;
  }
  // POTRF units in instances of their own: the register-resident factor up
  // to RPOTRF_MAX (its registers go to nothing else), and above it, in
  // graphs without GEMM or SYRK units, a left-looking one with the register-
  // resident factor's diagonal block and reciprocal substitution (compiled
  // into the full instance, or into one instance with the register-resident
  // factor, it spills); a unit of the wrong order is reported as a
  // breakdown at its first column rather than left unfactored
  if ((MODE == LI_POTRF || MODE == LI_POTRF_LL) && kind == K_POTRF) {
    const bool regs = __builtin_amdgcn_readfirstlane(d.m) <= RPOTRF_MAX;
    const int bad = MODE == LI_POTRF
                        ? (!regs ? 1
                           : d.tc == T_F32 ? run_potrf_regs<float>(d, lds)
                                           : run_potrf_regs<double>(d, lds))
                        : (regs ? 1
                           : d.tc == T_F32 ? run_potrf_ll<float>(d, lds)
                                           : run_potrf_ll<double>(d, lds));
    if (bad && threadIdx.x == 0 && d.matrix >= 0) {
      info[d.matrix] = d.row0 + bad;
      failed[d.matrix] = 1;
    }
  }
}

// Level executor: the workgroups of one level launch take the level's
// units through an atomic counter until the list is exhausted.
template <int MODE>
__global__ void __launch_bounds__(NT, (MODE == LI_LIGHT || MODE == LI_RHS) ? 4 : 1)
    dc_level_kernel(LevelArgs A) {
  extern __shared__ double lds[];
  __shared__ uint64_t s_idx;
  __shared__ int s_skip;
  const int tid = threadIdx.x;
  for (;;) {
    if (tid == 0)
      s_idx = __hip_atomic_fetch_add(A.counter, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    const uint64_t idx = uniform_u64(s_idx);
    if (idx >= (uint64_t)A.count) break;
    const uint64_t item = A.items[A.begin + idx];
    const int t = (int)(item >> 32);
    const int u = (int)(item & 0xffffffffu);
    const TaskDesc &d = A.desc[t];
    if (tid == 0) {
      s_skip = (d.matrix >= 0) ? A.failed[d.matrix] : 0;
      if (A.trace)
        atomicMin((unsigned long long *)&A.trace[3 * t], (unsigned long long)wall_clock64());
    }
    __syncthreads();
    if (!__builtin_amdgcn_readfirstlane(s_skip)) run_panel_unit<MODE>(d, u, lds, A.info, A.failed);
    if (A.trace && tid == 0) {
      atomicMax((unsigned long long *)&A.trace[3 * t + 1], (unsigned long long)wall_clock64());
      A.trace[3 * t + 2] = blockIdx.x;
    }
    __syncthreads();
  }
}

// Ready-queue executor, panel class: thread 0 pops a ready item (queue.h),
// the workgroup runs it, every thread's writes are released at agent scope,
// and thread 0 completes the item (releasing successors).  The worker
// leaves when every panel item has been claimed or the watchdog fired.
template <int MODE>
__global__ void __launch_bounds__(NT, (MODE == LI_FULL || MODE == LI_POTRF) ? 1 : 4)
    dc_queue_panel_kernel(QueueArgs A) {
  extern __shared__ double lds[];
  __shared__ uint64_t s_item;
  __shared__ int s_skip;
  const int tid = threadIdx.x;
  if (tid == 0) dcq::start_worker(&A.q, A.cls);
  for (;;) {
    if (tid == 0) s_item = dcq::pop_item(&A.q, A.cls);
    __syncthreads();
    const uint64_t item = uniform_u64(s_item);
    if (!item) break;
    const int64_t t = dcq::item_task(item);
    const int u = dcq::item_unit(item);
    const TaskDesc &d = A.desc[t];
    if (tid == 0) {
      s_skip = (d.matrix >= 0) ? A.failed[d.matrix] : 0;
      if (A.trace)
        atomicMin((unsigned long long *)&A.trace[3 * t], (unsigned long long)wall_clock64());
    }
    __syncthreads();
    if (!__builtin_amdgcn_readfirstlane(s_skip)) run_panel_unit<MODE>(d, u, lds, A.info, A.failed);
    if (A.trace && tid == 0) {
      atomicMax((unsigned long long *)&A.trace[3 * t + 1], (unsigned long long)wall_clock64());
      A.trace[3 * t + 2] = blockIdx.x;
    }
    dcq::DevAT::fence_rel();
    __syncthreads();
    if (tid == 0) dcq::complete_item(&A.q, t);
  }
}

// Fills x[i] = 2 i + 1 (a launch-path check with no waits).
__global__ void dc_fill_kernel(int64_t *x, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    x[i] = 2 * i + 1;
}

}  // namespace

extern "C" int dc_selftest(void *dev_ptr, int64_t n, void *stream) {
  if (!dev_ptr || n < 0) return -22;
  const int blocks = (int)((n + 255) / 256 < 1024 ? (n + 255) / 256 : 1024);
  if (blocks == 0) return 0;
  hipLaunchKernelGGL(dc_fill_kernel, dim3(blocks), dim3(256), 0, (hipStream_t)stream,
                     (int64_t *)dev_ptr, n);
  if (hipGetLastError() != hipSuccess) return -5;
  return hipStreamSynchronize((hipStream_t)stream) == hipSuccess ? 0 : -5;
}

int dcx_launch_level(const LevelArgs &args, int workers, size_t lds_bytes, int inst,
                     void *stream) {
  if (inst == LI_POTRF_LL)
    hipLaunchKernelGGL(dc_level_kernel<LI_POTRF_LL>, dim3(workers), dim3(NT), lds_bytes,
                       (hipStream_t)stream, args);
  else if (inst == LI_POTRF)
    hipLaunchKernelGGL(dc_level_kernel<LI_POTRF>, dim3(workers), dim3(NT), lds_bytes,
                       (hipStream_t)stream, args);
  else if (inst == LI_LIGHT)
    hipLaunchKernelGGL(dc_level_kernel<LI_LIGHT>, dim3(workers), dim3(NT), lds_bytes,
                       (hipStream_t)stream, args);
  else if (inst == LI_RHS)
    hipLaunchKernelGGL(dc_level_kernel<LI_RHS>, dim3(workers), dim3(NT), lds_bytes,
                       (hipStream_t)stream, args);
  else
    hipLaunchKernelGGL(dc_level_kernel<LI_FULL>, dim3(workers), dim3(NT), lds_bytes,
                       (hipStream_t)stream, args);
  return (int)hipGetLastError();
}

int dcx_launch_queue_panel(const QueueArgs &args, int workers, size_t lds_bytes, int inst,
                           void *stream) {
  if (inst == LI_LIGHT)
    hipLaunchKernelGGL(dc_queue_panel_kernel<LI_LIGHT>, dim3(workers), dim3(NT), lds_bytes,
                       (hipStream_t)stream, args);
  else if (inst == LI_RHS)
    hipLaunchKernelGGL(dc_queue_panel_kernel<LI_RHS>, dim3(workers), dim3(NT), lds_bytes,
                       (hipStream_t)stream, args);
  else
    hipLaunchKernelGGL(dc_queue_panel_kernel<LI_FULL>, dim3(workers), dim3(NT), lds_bytes,
                       (hipStream_t)stream, args);
  return (int)hipGetLastError();
}

int dcx_level_setup(void) {
  hipError_t e = hipSuccess;
  for (const void *f : {(const void *)dc_level_kernel<LI_FULL>,
                        (const void *)dc_level_kernel<LI_LIGHT>,
                        (const void *)dc_level_kernel<LI_RHS>,
                        (const void *)dc_level_kernel<LI_POTRF>,
                        (const void *)dc_level_kernel<LI_POTRF_LL>,
                        (const void *)dc_queue_panel_kernel<LI_FULL>,
                        (const void *)dc_queue_panel_kernel<LI_LIGHT>,
                        (const void *)dc_queue_panel_kernel<LI_RHS>})
    if (e == hipSuccess)
      e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize,
                              LDS_DOUBLES * (int)sizeof(double));
  return (int)e;
}

extern "C" int dc_executor_limits(int device, int64_t *out, int n) {
  // out: [lds_per_block_max, lds_per_cu_max, kernel_lds, kernel_scratch_per_lane,
  //       kernel_vgprs, occupancy_blocks_per_cu, max_threads_per_block]
  if (!out || n < 7) return -22;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) != hipSuccess) return -5;
  hipFuncAttributes fa;
  if (hipFuncGetAttributes(&fa, (const void *)dc_level_kernel<LI_FULL>) != hipSuccess) return -5;
  int nb = 0;
  hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, dc_level_kernel<LI_FULL>, NT,
                                               LDS_DOUBLES * sizeof(double));
  out[0] = (int64_t)prop.sharedMemPerBlock;
  out[1] = (int64_t)prop.maxSharedMemoryPerMultiProcessor;
  out[2] = (int64_t)fa.sharedSizeBytes;
  out[3] = (int64_t)fa.localSizeBytes;
  out[4] = (int64_t)fa.numRegs;
  out[5] = nb;
  out[6] = (int64_t)fa.maxThreadsPerBlock;
  return 0;
}

int dcx_queue_occupancy(size_t lds_bytes, int inst, int *blocks_per_cu) {
  int nb = 0;
  hipError_t e =
      inst == LI_LIGHT ? hipOccupancyMaxActiveBlocksPerMultiprocessor(
                             &nb, dc_queue_panel_kernel<LI_LIGHT>, NT, lds_bytes)
      : inst == LI_RHS ? hipOccupancyMaxActiveBlocksPerMultiprocessor(
                             &nb, dc_queue_panel_kernel<LI_RHS>, NT, lds_bytes)
                       : hipOccupancyMaxActiveBlocksPerMultiprocessor(
                             &nb, dc_queue_panel_kernel<LI_FULL>, NT, lds_bytes);
  *blocks_per_cu = nb;
  return (int)e;
}

int dcx_level_occupancy(size_t lds_bytes, int inst, int *blocks_per_cu) {
  int nb = 0;
  hipError_t e =
      inst == LI_POTRF_LL ? hipOccupancyMaxActiveBlocksPerMultiprocessor(
                             &nb, dc_level_kernel<LI_POTRF_LL>, NT, lds_bytes)
      : inst == LI_POTRF ? hipOccupancyMaxActiveBlocksPerMultiprocessor(
                             &nb, dc_level_kernel<LI_POTRF>, NT, lds_bytes)
      : inst == LI_LIGHT ? hipOccupancyMaxActiveBlocksPerMultiprocessor(
                             &nb, dc_level_kernel<LI_LIGHT>, NT, lds_bytes)
      : inst == LI_RHS ? hipOccupancyMaxActiveBlocksPerMultiprocessor(
                             &nb, dc_level_kernel<LI_RHS>, NT, lds_bytes)
                       : hipOccupancyMaxActiveBlocksPerMultiprocessor(
                             &nb, dc_level_kernel<LI_FULL>, NT, lds_bytes);
  *blocks_per_cu = nb;
  return (int)e;
}

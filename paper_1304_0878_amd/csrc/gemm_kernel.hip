// GEMM/SYRK work units of the level executor (the trailing updates of the
// right-looking tiled Cholesky), in FP64, FP32 and BF16 input precision.
//
// One workgroup of 512 threads (eight 64-wide waves, two per SIMD) computes
// one 128x128 output block: C -= A B^T with A (128 x K) and B (128 x K) rows
// K-contiguous.  Waves form a 2 x 4 grid of 64 x 32 tiles.  Operands are
// staged through LDS in K chunks, double buffered, with padded row strides so
// that the fragment reads of 16 consecutive rows fall in distinct banks.
//
//   FP64: 4x4x4 (4-block) FP64 MFMA, C pre-loaded (negated) into the
//         accumulators so the epilogue is a plain store.
//   FP32: 16x16x4 FP32 MFMA, FP32 accumulation; result subtracted from an
//         FP32 or FP64 C.
//   BF16: 16x16x32 BF16 MFMA on BF16 inputs, FP32 accumulation; result
//         subtracted from an FP32 or FP64 C.
// SYRK units on the diagonal write only the lower triangle.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "exec_abi.h"
#include "queue_dev.h"

using namespace dcx;

namespace {

constexpr int GT = 512;   // threads per workgroup

typedef __attribute__((address_space(1))) double gdouble;
typedef __attribute__((address_space(1))) float gfloat;
typedef __attribute__((address_space(1))) __bf16 gbf16;
typedef double dvec2 __attribute__((ext_vector_type(2)));
typedef float fvec4 __attribute__((ext_vector_type(4)));
typedef __bf16 bvec8 __attribute__((ext_vector_type(8)));
typedef __attribute__((address_space(1))) dvec2 gdvec2;
typedef __attribute__((address_space(1))) fvec4 gfvec4;
typedef __attribute__((address_space(1))) bvec8 gbvec8;
template <typename T> using gp = __attribute__((address_space(1))) T *;

// ------------------------------------------------------------------ FP64
//
// FP64 units run in their own kernel, one 512-thread workgroup per CU made
// of two halves that each compute one unit of the same task (four waves in
// a 2 x 2 grid of 64 x 64 tiles): two waves per SIMD, yet a single
// workgroup per CU, so the kernel never takes the CUs the panel kernel was
// left.  16x16x4 FP64 MFMA (lane l
// supplies A[l%16][l/16] and B^T[l/16][l%16]; result element e of lane l is
// D[l/16 + 4e][l%16]).  K chunks of 16 are staged in LDS, double buffered,
// with an odd row stride (17 doubles): the 16 lanes that read one fragment
// at a time read 16 rows at one column, which then fall in distinct banks.
// C is pre-loaded negated into the accumulators, so the epilogue is a plain
// store of the negation.

constexpr int GT64 = 512;                     // two halves of 256 threads
constexpr int KC64 = 16;
constexpr int S64 = KC64 + 1;                 // doubles per LDS row
constexpr int STAGE64 = 2 * GEMM_UNIT * S64;  // A and B of one stage

typedef double dvec4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ dvec4 mfma16(double a, double b, dvec4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Global memory is reached through buffer resources that span exactly the
// unit's rows of each operand: a per-lane 32-bit offset plus a wave-uniform
// scalar offset per row group, so addressing costs one VGPR per operand, and
// an access outside the span reads zero or is dropped instead of faulting.
// The row span of one unit is below 4 GiB because leading dimensions are
// limited at registration.
__device__ __forceinline__ uint64_t uniform_u64(uint64_t v) {
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
  return ((uint64_t)hi << 32) | lo;
}

typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ __amdgpu_buffer_rsrc_t span_rsrc(const void *base, int64_t rows,
                                                            int64_t ld, int64_t cols,
                                                            int esize = 8) {
  const int64_t bytes = rows > 0 ? ((rows - 1) * ld + cols) * esize : 0;
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), 0, (int)(uint32_t)bytes,
                                           0x00020000);
}
__device__ __forceinline__ double bload(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
}
__device__ __forceinline__ void bstore(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff,
                                       double v) {
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, voff, soff, 0);
}
typedef float fvec2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ float bloadf(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
}
__device__ __forceinline__ fvec2 bloadf2(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
  return __builtin_bit_cast(fvec2, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
}
__device__ __forceinline__ void bstoref(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff,
                                        float v) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned int, v), r, voff, soff, 0);
}

// Ragged units (M or N below the unit size, K not a multiple of the chunk)
// clamp row and column indices, so every load stays inside the unit: rows
// past M (N) only feed output rows (columns) that are not stored, and
// columns past K are selected to zero.  dlim is the largest column - row
// offset that is stored: 0 for the lower-triangular diagonal units of SYRK,
// otherwise unbounded.  It depends on the unit, so the comparison stays
// inside the unit loop instead of being hoisted into 64 saved masks.
template <bool FULL>
__device__ __forceinline__ void block_f64(void *C, int64_t ldc, const void *A, int64_t lda,
                                          const void *B, int64_t ldb, int M, int N, int K,
                                          int dlim, double *lds, int tid) {
  const int lane = tid & 63, w = tid >> 6;
  const int wr = w >> 1, wc = w & 1;
  const int l16 = lane & 15, kq = lane >> 4;
  const int r0 = 64 * wr + kq, c0 = 64 * wc + l16;  // element (i, j, e) at r0 + 16i + 4e, c0 + 16j
  const __amdgpu_buffer_rsrc_t rc = span_rsrc(C, M, ldc, N);
  const __amdgpu_buffer_rsrc_t ra_ = span_rsrc(A, M, lda, K);
  const __amdgpu_buffer_rsrc_t rb_ = span_rsrc(B, N, ldb, K);
  const uint32_t cld = (uint32_t)ldc * 8;
  dvec4 acc[4][4];
  {
    const uint32_t cv = FULL ? ((uint32_t)r0 * (uint32_t)ldc + c0) * 8 : 0;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          if (FULL) {
            acc[i][j][e] = -bload(rc, cv + 128 * j, (16 * i + 4 * e) * cld);
          } else {
            const uint32_t row = min(r0 + 16 * i + 4 * e, M - 1);
            const uint32_t col = min(c0 + 16 * j, N - 1);
            acc[i][j][e] = -bload(rc, (row * (uint32_t)ldc + col) * 8, 0);
          }
        }
  }
  // loader: thread -> rows tid/16 + 16 jj, column tid%16 of the chunk
  const int lrow = tid >> 4, lcol = tid & 15;
  const uint32_t ald = (uint32_t)lda * 8, bld = (uint32_t)ldb * 8;
  const uint32_t av = (uint32_t)lrow * ald + lcol * 8, bv = (uint32_t)lrow * bld + lcol * 8;
  double ra[8], rb[8];
  auto gload = [&](int k0) {
    if (FULL) {
#pragma unroll
      for (int jj = 0; jj < 8; ++jj) {
        ra[jj] = bload(ra_, av, 16 * jj * ald + k0 * 8);
        rb[jj] = bload(rb_, bv, 16 * jj * bld + k0 * 8);
      }
    } else {
      const uint32_t kc = min(k0 + lcol, K - 1);
#pragma unroll
      for (int jj = 0; jj < 8; ++jj) {
        const uint32_t ar = min(lrow + 16 * jj, M - 1), br = min(lrow + 16 * jj, N - 1);
        ra[jj] = bload(ra_, (ar * (uint32_t)lda + kc) * 8, 0);
        rb[jj] = bload(rb_, (br * (uint32_t)ldb + kc) * 8, 0);
      }
      if (k0 + lcol >= K) {
#pragma unroll
        for (int jj = 0; jj < 8; ++jj) ra[jj] = rb[jj] = 0.0;
      }
    }
  };
  auto sstore = [&](int st) {
    double *As = lds + st * STAGE64;
    double *Bs = As + GEMM_UNIT * S64;
#pragma unroll
    for (int jj = 0; jj < 8; ++jj) {
      As[(lrow + 16 * jj) * S64 + lcol] = ra[jj];
      Bs[(lrow + 16 * jj) * S64 + lcol] = rb[jj];
    }
  };
  const int nst = (K + KC64 - 1) / KC64;
  gload(0);
  sstore(0);
  __syncthreads();
  for (int st = 0; st < nst; ++st) {
    const int cur = st & 1;
    if (st + 1 < nst) gload((st + 1) * KC64);
    const double *As = lds + cur * STAGE64;
    const double *Bs = As + GEMM_UNIT * S64;
#pragma unroll
    for (int ks = 0; ks < KC64 / 4; ++ks) {
      const int kk = 4 * ks + kq;
      double a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = As[(64 * wr + 16 * i + l16) * S64 + kk];
#pragma unroll
      for (int j = 0; j < 4; ++j) b[j] = Bs[(64 * wc + 16 * j + l16) * S64 + kk];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = mfma16(a[i], b[j], acc[i][j]);
    }
    if (st + 1 < nst) sstore(cur ^ 1);
    __syncthreads();
  }
  const int dbase = c0 - r0;
  const uint32_t cv = ((uint32_t)r0 * (uint32_t)ldc + c0) * 8;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int row = r0 + 16 * i + 4 * e, col = c0 + 16 * j;
        if ((FULL || (row < M && col < N)) && dbase + 16 * (j - i) - 4 * e <= dlim)
          bstore(rc, cv + 128 * j, (16 * i + 4 * e) * cld, -acc[i][j][e]);
      }
}

// FP32 inputs in the same two-half workgroup: the FP64 block's structure
// with 16x16x4 FP32 MFMA (result element e of lane l is D[4(l/16) + e][l%16]),
// K chunks of 32 floats in LDS with a row stride of 34 floats (the 32 lanes
// of one half-wave read 16 rows at two adjacent columns: banks 2*row + kq are
// distinct), two floats per lane and row in each global load, FP32
// accumulation, and C <- C - acc in C's own precision at the end (an FP64
// tile keeps its FP64 value; only the product is FP32).
constexpr int KCF = 32;
constexpr int SF = KCF + 2;                   // floats per LDS row
constexpr int STAGEF = 2 * GEMM_UNIT * SF;    // A and B of one stage
static_assert(2 * STAGEF * 4 <= 2 * STAGE64 * 8, "FP32 stages fit a half's LDS");

template <bool FULL, typename TOUT>
__device__ __forceinline__ void block_f32p(void *C, int64_t ldc, const void *A, int64_t lda,
                                           const void *B, int64_t ldb, int M, int N, int K,
                                           int dlim, float *lds, int tid) {
  const int lane = tid & 63, w = tid >> 6;
  const int wr = w >> 1, wc = w & 1;
  const int l16 = lane & 15, kq = lane >> 4;
  const __amdgpu_buffer_rsrc_t rc = span_rsrc(C, M, ldc, N, (int)sizeof(TOUT));
  const __amdgpu_buffer_rsrc_t ra_ = span_rsrc(A, M, lda, K, 4);
  const __amdgpu_buffer_rsrc_t rb_ = span_rsrc(B, N, ldb, K, 4);
  fvec4 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = (fvec4){0.f, 0.f, 0.f, 0.f};
  // loader: thread -> rows tid/16 + 16 jj, columns 2(tid%16), +1 of the chunk
  const int lrow = tid >> 4, lcol = (tid & 15) * 2;
  const uint32_t ald = (uint32_t)lda * 4, bld = (uint32_t)ldb * 4;
  const uint32_t av = (uint32_t)lrow * ald + lcol * 4, bv = (uint32_t)lrow * bld + lcol * 4;
  fvec2 ra[8], rb[8];
  auto gload = [&](int k0) {
    if (FULL) {
#pragma unroll
      for (int jj = 0; jj < 8; ++jj) {
        ra[jj] = bloadf2(ra_, av, 16 * jj * ald + k0 * 4);
        rb[jj] = bloadf2(rb_, bv, 16 * jj * bld + k0 * 4);
      }
    } else {
#pragma unroll
      for (int jj = 0; jj < 8; ++jj) {
        const uint32_t ar = min(lrow + 16 * jj, M - 1), br = min(lrow + 16 * jj, N - 1);
#pragma unroll
        for (int e = 0; e < 2; ++e) {
          const int k = k0 + lcol + e;
          const uint32_t kc = min(k, K - 1);
          const float x = bloadf(ra_, (ar * (uint32_t)lda + kc) * 4, 0);
          const float y = bloadf(rb_, (br * (uint32_t)ldb + kc) * 4, 0);
          ra[jj][e] = k < K ? x : 0.f;
          rb[jj][e] = k < K ? y : 0.f;
        }
      }
    }
  };
  auto sstore = [&](int st) {
    float *As = lds + st * STAGEF;
    float *Bs = As + GEMM_UNIT * SF;
#pragma unroll
    for (int jj = 0; jj < 8; ++jj) {
      *(fvec2 *)(As + (lrow + 16 * jj) * SF + lcol) = ra[jj];
      *(fvec2 *)(Bs + (lrow + 16 * jj) * SF + lcol) = rb[jj];
    }
  };
  const int nst = (K + KCF - 1) / KCF;
  gload(0);
  sstore(0);
  __syncthreads();
  for (int st = 0; st < nst; ++st) {
    const int cur = st & 1;
    if (st + 1 < nst) gload((st + 1) * KCF);
    const float *As = lds + cur * STAGEF;
    const float *Bs = As + GEMM_UNIT * SF;
#pragma unroll
    for (int ks = 0; ks < KCF / 4; ++ks) {
      const int kk = 4 * ks + kq;
      float a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = As[(64 * wr + 16 * i + l16) * SF + kk];
#pragma unroll
      for (int j = 0; j < 4; ++j) b[j] = Bs[(64 * wc + 16 * j + l16) * SF + kk];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    if (st + 1 < nst) sstore(cur ^ 1);
    __syncthreads();
  }
  const int r0 = 64 * wr + 4 * kq, c0 = 64 * wc + l16;   // element (i, j, e) at r0 + 16i + e, c0 + 16j
  const int dbase = c0 - r0;
  constexpr uint32_t es = sizeof(TOUT);
  const uint32_t cld = (uint32_t)ldc * es;
  const uint32_t cv = ((uint32_t)r0 * (uint32_t)ldc + c0) * es;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int row = r0 + 16 * i + e, col = c0 + 16 * j;
        if ((FULL || (row < M && col < N)) && dbase + 16 * (j - i) - e <= dlim) {
          const uint32_t so = (16 * i + e) * cld;
          if (sizeof(TOUT) == 8) {
            const double v = bload(rc, cv + 16 * es * j, so);
            bstore(rc, cv + 16 * es * j, so, v - (double)acc[i][j][e]);
          } else {
            const float v = bloadf(rc, cv + 16 * es * j, so);
            bstoref(rc, cv + 16 * es * j, so, v - acc[i][j][e]);
          }
        }
      }
}

// ------------------------------------------------------------ BF16 inputs

// Epilogue of the BF16 path: 16x16 MFMA output layout
// (lane l holds rows 4(l/16)+e, column l%16 of its 16x16 tile).
template <typename TOUT>
__device__ __forceinline__ void store_lowp(gp<TOUT> __restrict__ C, int64_t ldc, int M, int N,
                                           bool lower_only, const fvec4 (&acc)[4][2]) {
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wr = w >> 2, wc = w & 3;
  const int l16 = lane & 15, kq = lane >> 4;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int row = 64 * wr + 16 * i + 4 * kq + e;
        const int col = 32 * wc + 16 * c + l16;
        if (row < M && col < N && (!lower_only || col <= row)) {
          gp<TOUT> p = C + (int64_t)row * ldc + col;
          *p = *p - (TOUT)acc[i][c][e];
        }
      }
}

constexpr int KC16 = 64;
constexpr int S16 = KC16 + 8;                 // bf16 per LDS row
constexpr int STAGE16 = 2 * GEMM_UNIT * S16;

template <typename TOUT>
__device__ __forceinline__ void block_bf16(gp<TOUT> __restrict__ C, int64_t ldc,
                                           const gbf16 *__restrict__ A, int64_t lda,
                                           const gbf16 *__restrict__ B, int64_t ldb, int M,
                                           int N, int K, bool lower_only, __bf16 *lds) {
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wr = w >> 2, wc = w & 3;
  const int l16 = lane & 15, kq = lane >> 4;
  fvec4 acc[4][2];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int c = 0; c < 2; ++c) acc[i][c] = (fvec4){0.f, 0.f, 0.f, 0.f};
  // loader: 8 threads per row (eight bf16 each), 64 rows per pass, 2 passes
  const int lrow = tid >> 3, lk = (tid & 7) * 8;
  const bool fast = M == GEMM_UNIT && N == GEMM_UNIT && (K % KC16) == 0 &&
                    (((uintptr_t)A | (uintptr_t)B) & 15) == 0 && ((lda | ldb) & 7) == 0;
  bvec8 ra[2], rb[2];
  auto gload = [&](int k0) {
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int row = lrow + 64 * j;
      if (fast) {
        ra[j] = *(const gbvec8 *)(A + (int64_t)row * lda + k0 + lk);
        rb[j] = *(const gbvec8 *)(B + (int64_t)row * ldb + k0 + lk);
      } else {
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const int k = k0 + lk + e;
          ra[j][e] = (row < M && k < K) ? A[(int64_t)row * lda + k] : (__bf16)0.f;
          rb[j][e] = (row < N && k < K) ? B[(int64_t)row * ldb + k] : (__bf16)0.f;
        }
      }
    }
  };
  auto sstore = [&](int st) {
    __bf16 *As = lds + st * STAGE16;
    __bf16 *Bs = As + GEMM_UNIT * S16;
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      *(bvec8 *)(As + (lrow + 64 * j) * S16 + lk) = ra[j];
      *(bvec8 *)(Bs + (lrow + 64 * j) * S16 + lk) = rb[j];
    }
  };
  const int nst = (K + KC16 - 1) / KC16;
  gload(0);
  sstore(0);
  __syncthreads();
  for (int st = 0; st < nst; ++st) {
    const int cur = st & 1;
    if (st + 1 < nst) gload((st + 1) * KC16);
    const __bf16 *As = lds + cur * STAGE16;
    const __bf16 *Bs = As + GEMM_UNIT * S16;
#pragma unroll
    for (int ks = 0; ks < KC16 / 32; ++ks) {
      const int kk = 32 * ks + 8 * kq;
      bvec8 a[4], b[2];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = *(const bvec8 *)(As + (64 * wr + 16 * i + l16) * S16 + kk);
#pragma unroll
      for (int c = 0; c < 2; ++c) b[c] = *(const bvec8 *)(Bs + (32 * wc + 16 * c + l16) * S16 + kk);
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int c = 0; c < 2; ++c)
          acc[i][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[c], acc[i][c], 0, 0, 0);
    }
    if (st + 1 < nst) sstore(cur ^ 1);
    __syncthreads();
  }
  store_lowp<TOUT>(C, ldc, M, N, lower_only, acc);
}

// --------------------------------------------------------- unit dispatch

// Position of a unit in its task: the output block (p, q) of 128 x 128, its
// extent, and for SYRK whether it lies on the diagonal (lower half only).
struct UnitBlock {
  int M, N;
  bool lower_only;
  const void *a, *b;
  int64_t lda, ldb, coff;
};

__device__ __forceinline__ UnitBlock unit_block(const TaskDesc &d, int unit, int esize) {
  int p, q;
  UnitBlock u;
  if (d.kind == K_SYRK) {
    p = 0;
    while ((p + 1) * (p + 2) / 2 <= unit) ++p;
    q = unit - p * (p + 1) / 2;
    u.M = min(GEMM_UNIT, d.m - p * GEMM_UNIT);
    u.N = min(GEMM_UNIT, d.m - q * GEMM_UNIT);
    u.lower_only = p == q;
  } else {
    const int qn = (d.n + GEMM_UNIT - 1) / GEMM_UNIT;
    p = unit / qn;
    q = unit % qn;
    u.M = min(GEMM_UNIT, d.m - p * GEMM_UNIT);
    u.N = min(GEMM_UNIT, d.n - q * GEMM_UNIT);
    u.lower_only = false;
  }
  const int r0 = p * GEMM_UNIT, c0 = q * GEMM_UNIT;
  // SYRK reads both operands from its one input
  u.lda = d.lda;
  u.ldb = d.kind == K_SYRK ? d.lda : d.ldb;
  u.a = (const char *)d.a + (int64_t)r0 * d.lda * esize;
  u.b = (const char *)(d.kind == K_SYRK ? d.a : d.b) + (int64_t)c0 * u.ldb * esize;
  u.coff = (int64_t)r0 * d.ldc + c0;
  return u;
}

template <int TA>
__device__ __forceinline__ void run_unit_pair(const TaskDesc &d, int unit, double *lds, int tid) {
  const UnitBlock u = unit_block(d, unit, TA == T_F64 ? 8 : 4);
  // buffer resources must sit in scalar registers: make the wave-uniform
  // unit fields provably uniform so no per-lane resource loop is generated
  auto su64 = [](const void *p) { return (void *)uniform_u64((uint64_t)p); };
  auto s32 = [](int64_t v) { return (int64_t)(int)__builtin_amdgcn_readfirstlane((int)v); };
  void *C = su64((char *)d.c + u.coff * (d.tc == T_F64 ? 8 : 4));
  const void *a = su64(u.a), *b = su64(u.b);
  const int64_t ldc = s32(d.ldc), lda = s32(u.lda), ldb = s32(u.ldb);
  const int M = __builtin_amdgcn_readfirstlane(u.M), N = __builtin_amdgcn_readfirstlane(u.N);
  const int K = __builtin_amdgcn_readfirstlane(d.k);
  const int dlim = __builtin_amdgcn_readfirstlane(u.lower_only ? 0 : GEMM_UNIT);
  const bool full = M == GEMM_UNIT && N == GEMM_UNIT;
  if constexpr (TA == T_F64) {
    if (full && K % KC64 == 0)
      block_f64<true>(C, ldc, a, lda, b, ldb, M, N, K, dlim, lds, tid);
    else
      block_f64<false>(C, ldc, a, lda, b, ldb, M, N, K, dlim, lds, tid);
  } else {
    // FP32 inputs: two-float loads need 8-byte aligned rows
    const bool f2 = full && K % KCF == 0 && ((lda | ldb) & 1) == 0 &&
                    (((uintptr_t)a | (uintptr_t)b) & 7) == 0;
    float *fl = (float *)lds;
    if (__builtin_amdgcn_readfirstlane(d.tc) == T_F64) {
      if (f2) block_f32p<true, double>(C, ldc, a, lda, b, ldb, M, N, K, dlim, fl, tid);
      else block_f32p<false, double>(C, ldc, a, lda, b, ldb, M, N, K, dlim, fl, tid);
    } else {
      if (f2) block_f32p<true, float>(C, ldc, a, lda, b, ldb, M, N, K, dlim, fl, tid);
      else block_f32p<false, float>(C, ldc, a, lda, b, ldb, M, N, K, dlim, fl, tid);
    }
  }
}

__device__ __forceinline__ void run_unit_lowp(const TaskDesc &d, int unit, double *lds) {
  const UnitBlock u = unit_block(d, unit, 2);
  const gbf16 *A = (const gbf16 *)u.a, *B = (const gbf16 *)u.b;
  if (d.tc == T_F64)
    block_bf16<double>((gdouble *)d.c + u.coff, d.ldc, A, u.lda, B, u.ldb, u.M, u.N, d.k,
                        u.lower_only, (__bf16 *)lds);
  else
    block_bf16<float>((gfloat *)d.c + u.coff, d.ldc, A, u.lda, B, u.ldb, u.M, u.N, d.k,
                       u.lower_only, (__bf16 *)lds);
}

// Persistent loop of a GEMM kernel: take units from the level's counter
// until the list is exhausted.  The failure flag of the unit's matrix can
// be set during the level by a POTRF unit of the panel kernel, so one thread
// reads it and the workgroup takes the decision from LDS after a barrier.
template <typename RUN>
__device__ __forceinline__ void unit_loop(const LevelArgs &A, double *lds, RUN run) {
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
    if (!__builtin_amdgcn_readfirstlane(s_skip)) run(d, u, lds);
    if (A.trace && tid == 0) {
      atomicMax((unsigned long long *)&A.trace[3 * t + 1], (unsigned long long)wall_clock64());
      A.trace[3 * t + 2] = blockIdx.x;
    }
    __syncthreads();
  }
}

// Ready-queue loop of a GEMM kernel: thread 0 pops a ready item of the
// launch's class (queue.h), the workgroup runs it, every thread's writes are
// released at agent scope and thread 0 completes the item, which releases
// the successors whose last dependency it was.
template <typename RUN>
__device__ __forceinline__ void queue_loop(const QueueArgs &A, double *lds, RUN run) {
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
    if (!__builtin_amdgcn_readfirstlane(s_skip)) run(d, u, lds);
    if (A.trace && tid == 0) {
      atomicMax((unsigned long long *)&A.trace[3 * t + 1], (unsigned long long)wall_clock64());
      A.trace[3 * t + 2] = blockIdx.x;
    }
    dcq::DevAT::fence_rel();
    __syncthreads();
    if (tid == 0) dcq::complete_item(&A.q, t);
  }
}

// One work item of the two-half kernel: units u0 and u0 + 1 of one task, one
// per half.  Both have the task's K and so pass the same number of
// workgroup barriers; a half without a unit (odd unit count) only passes
// them.  One kernel instance per input type (FP64 or FP32), so each keeps
// its own register allocation.
template <int TA>
__device__ __forceinline__ void run_pair(const TaskDesc &d, int u0, double *lds) {
  const int half = threadIdx.x >> 8, tid = threadIdx.x & 255;
  const int unit = u0 + half;
  if (unit < __builtin_amdgcn_readfirstlane(d.nunits)) {
    run_unit_pair<TA>(d, unit, lds + half * 2 * STAGE64, tid);
  } else {
    constexpr int kc = TA == T_F64 ? KC64 : KCF;
    const int nst = (__builtin_amdgcn_readfirstlane(d.k) + kc - 1) / kc;
    for (int i = 0; i <= nst; ++i) __syncthreads();
  }
}
template <int TA>
__global__ void __launch_bounds__(GT64, 1) dc_gemm_kernel(LevelArgs A) {
  extern __shared__ double lds[];
  unit_loop(A, lds, [](const TaskDesc &d, int u, double *l) { run_pair<TA>(d, u, l); });
}

// GEMM/SYRK units with BF16 inputs.
__global__ void __launch_bounds__(GT, 1) dc_gemm_lowp_kernel(LevelArgs A) {
  extern __shared__ double lds[];
  unit_loop(A, lds, [](const TaskDesc &d, int u, double *l) { run_unit_lowp(d, u, l); });
}

template <int TA>
__global__ void __launch_bounds__(GT64, 1) dc_queue_gemm_kernel(QueueArgs A) {
  extern __shared__ double lds[];
  queue_loop(A, lds, [](const TaskDesc &d, int u, double *l) { run_pair<TA>(d, u, l); });
}

__global__ void __launch_bounds__(GT, 1) dc_queue_gemm_lowp_kernel(QueueArgs A) {
  extern __shared__ double lds[];
  queue_loop(A, lds, [](const TaskDesc &d, int u, double *l) { run_unit_lowp(d, u, l); });
}

constexpr int GEMM_KERNEL_LDS = 2 * 2 * STAGE64 * (int)sizeof(double);   // two halves
constexpr int GEMM_LOWP_LDS = 2 * STAGE16 * 2;   // two stages of BF16 A and B
static_assert(GEMM_KERNEL_LDS + 64 <= 160 * 1024, "FP64 workgroup LDS");

}  // namespace

int dcx_launch_gemm(const LevelArgs &args, int workers, int ta, void *stream) {
  if (ta == T_F64)
    hipLaunchKernelGGL(dc_gemm_kernel<T_F64>, dim3(workers), dim3(GT64), GEMM_KERNEL_LDS,
                       (hipStream_t)stream, args);
  else
    hipLaunchKernelGGL(dc_gemm_kernel<T_F32>, dim3(workers), dim3(GT64), GEMM_KERNEL_LDS,
                       (hipStream_t)stream, args);
  return (int)hipGetLastError();
}

int dcx_launch_gemm_lowp(const LevelArgs &args, int workers, void *stream) {
  hipLaunchKernelGGL(dc_gemm_lowp_kernel, dim3(workers), dim3(GT), GEMM_LOWP_LDS,
                     (hipStream_t)stream, args);
  return (int)hipGetLastError();
}

int dcx_launch_queue_gemm(const QueueArgs &args, int workers, void *stream) {
  if (args.cls == dcq::CL_G64)
    hipLaunchKernelGGL(dc_queue_gemm_kernel<T_F64>, dim3(workers), dim3(GT64), GEMM_KERNEL_LDS,
                       (hipStream_t)stream, args);
  else if (args.cls == dcq::CL_G32)
    hipLaunchKernelGGL(dc_queue_gemm_kernel<T_F32>, dim3(workers), dim3(GT64), GEMM_KERNEL_LDS,
                       (hipStream_t)stream, args);
  else
    hipLaunchKernelGGL(dc_queue_gemm_lowp_kernel, dim3(workers), dim3(GT), GEMM_LOWP_LDS,
                       (hipStream_t)stream, args);
  return (int)hipGetLastError();
}

int dcx_gemm_setup(void) {
  hipError_t e = hipFuncSetAttribute((const void *)dc_gemm_kernel<T_F64>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, GEMM_KERNEL_LDS);
  if (e == hipSuccess)
    e = hipFuncSetAttribute((const void *)dc_gemm_kernel<T_F32>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, GEMM_KERNEL_LDS);
  if (e == hipSuccess)
    e = hipFuncSetAttribute((const void *)dc_gemm_lowp_kernel,
                            hipFuncAttributeMaxDynamicSharedMemorySize, GEMM_LOWP_LDS);
  if (e == hipSuccess)
    e = hipFuncSetAttribute((const void *)dc_queue_gemm_kernel<T_F64>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, GEMM_KERNEL_LDS);
  if (e == hipSuccess)
    e = hipFuncSetAttribute((const void *)dc_queue_gemm_kernel<T_F32>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, GEMM_KERNEL_LDS);
  if (e == hipSuccess)
    e = hipFuncSetAttribute((const void *)dc_queue_gemm_lowp_kernel,
                            hipFuncAttributeMaxDynamicSharedMemorySize, GEMM_LOWP_LDS);
  return (int)e;
}

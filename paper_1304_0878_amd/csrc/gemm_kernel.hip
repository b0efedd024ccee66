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

__device__ __forceinline__ double mfma44(double a, double b, double c) {
  return __builtin_amdgcn_mfma_f64_4x4x4f64(a, b, c, 0, 0, 0);
}

// ------------------------------------------------------------------ FP64

constexpr int KC64 = 32;
constexpr int S64 = KC64 + 2;                 // doubles per LDS row
constexpr int STAGE64 = 2 * GEMM_UNIT * S64;  // A and B of one stage

__device__ __forceinline__ void block_f64(gdouble *__restrict__ C, int64_t ldc,
                                          const gdouble *__restrict__ A, int64_t lda,
                                          const gdouble *__restrict__ B, int64_t ldb, int M,
                                          int N, int K, bool lower_only, double *lds) {
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wr = w >> 2, wc = w & 3;
  const int l16 = lane & 15, blk = l16 >> 2, kq = lane >> 4, n4 = lane & 3;
  double acc[4][2][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const int row = 64 * wr + 16 * i + 4 * blk + kq;
        const int col = 32 * wc + 16 * c + 4 * ((blk + s) & 3) + n4;
        const bool ok = row < M && col < N && (!lower_only || col <= row);
        acc[i][c][s] = ok ? -C[(int64_t)row * ldc + col] : 0.0;
      }
  // loader: 16 threads per row (16-byte pairs), 32 rows per pass, 4 passes
  const int lrow = tid >> 4, lkp = (tid & 15) * 2;
  const bool fast = M == GEMM_UNIT && N == GEMM_UNIT && (K % KC64) == 0 &&
                    (((uintptr_t)A | (uintptr_t)B) & 15) == 0 && ((lda | ldb) & 1) == 0;
  dvec2 ra[4], rb[4];
  auto gload = [&](int k0) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int row = lrow + 32 * j;
      if (fast) {
        ra[j] = *(const gdvec2 *)(A + (int64_t)row * lda + k0 + lkp);
        rb[j] = *(const gdvec2 *)(B + (int64_t)row * ldb + k0 + lkp);
      } else {
        const int k = k0 + lkp;
        const gdouble *ap = A + (int64_t)row * lda + k;
        const gdouble *bp = B + (int64_t)row * ldb + k;
        ra[j].x = (row < M && k < K) ? ap[0] : 0.0;
        ra[j].y = (row < M && k + 1 < K) ? ap[1] : 0.0;
        rb[j].x = (row < N && k < K) ? bp[0] : 0.0;
        rb[j].y = (row < N && k + 1 < K) ? bp[1] : 0.0;
      }
    }
  };
  auto sstore = [&](int st) {
    double *As = lds + st * STAGE64;
    double *Bs = As + GEMM_UNIT * S64;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      *(dvec2 *)(As + (lrow + 32 * j) * S64 + lkp) = ra[j];
      *(dvec2 *)(Bs + (lrow + 32 * j) * S64 + lkp) = rb[j];
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
      double a[4], b[2][4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = As[(64 * wr + 16 * i + l16) * S64 + kk];
#pragma unroll
      for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int s = 0; s < 4; ++s)
          b[c][s] = Bs[(32 * wc + 16 * c + 4 * ((blk + s) & 3) + n4) * S64 + kk];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int c = 0; c < 2; ++c)
#pragma unroll
          for (int s = 0; s < 4; ++s) acc[i][c][s] = mfma44(a[i], b[c][s], acc[i][c][s]);
    }
    if (st + 1 < nst) sstore(cur ^ 1);
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const int row = 64 * wr + 16 * i + 4 * blk + kq;
        const int col = 32 * wc + 16 * c + 4 * ((blk + s) & 3) + n4;
        if (row < M && col < N && (!lower_only || col <= row))
          C[(int64_t)row * ldc + col] = -acc[i][c][s];
      }
}

// ------------------------------------------------- FP32 and BF16 inputs

// Epilogue shared by the low-precision paths: 16x16 MFMA output layout
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

constexpr int KC32 = 32;
constexpr int S32 = KC32 + 4;                 // floats per LDS row
constexpr int STAGE32 = 2 * GEMM_UNIT * S32;

template <typename TOUT>
__device__ __forceinline__ void block_f32(gp<TOUT> __restrict__ C, int64_t ldc,
                                          const gfloat *__restrict__ A, int64_t lda,
                                          const gfloat *__restrict__ B, int64_t ldb, int M,
                                          int N, int K, bool lower_only, float *lds) {
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wr = w >> 2, wc = w & 3;
  const int l16 = lane & 15, kq = lane >> 4;
  fvec4 acc[4][2];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int c = 0; c < 2; ++c) acc[i][c] = (fvec4){0.f, 0.f, 0.f, 0.f};
  // loader: 8 threads per row (four floats each), 64 rows per pass, 2 passes
  const int lrow = tid >> 3, lk = (tid & 7) * 4;
  const bool fast = M == GEMM_UNIT && N == GEMM_UNIT && (K % KC32) == 0 &&
                    (((uintptr_t)A | (uintptr_t)B) & 15) == 0 && ((lda | ldb) & 3) == 0;
  fvec4 ra[2], rb[2];
  auto gload = [&](int k0) {
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int row = lrow + 64 * j;
      if (fast) {
        ra[j] = *(const gfvec4 *)(A + (int64_t)row * lda + k0 + lk);
        rb[j] = *(const gfvec4 *)(B + (int64_t)row * ldb + k0 + lk);
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int k = k0 + lk + e;
          ra[j][e] = (row < M && k < K) ? A[(int64_t)row * lda + k] : 0.f;
          rb[j][e] = (row < N && k < K) ? B[(int64_t)row * ldb + k] : 0.f;
        }
      }
    }
  };
  auto sstore = [&](int st) {
    float *As = lds + st * STAGE32;
    float *Bs = As + GEMM_UNIT * S32;
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      *(fvec4 *)(As + (lrow + 64 * j) * S32 + lk) = ra[j];
      *(fvec4 *)(Bs + (lrow + 64 * j) * S32 + lk) = rb[j];
    }
  };
  const int nst = (K + KC32 - 1) / KC32;
  gload(0);
  sstore(0);
  __syncthreads();
  for (int st = 0; st < nst; ++st) {
    const int cur = st & 1;
    if (st + 1 < nst) gload((st + 1) * KC32);
    const float *As = lds + cur * STAGE32;
    const float *Bs = As + GEMM_UNIT * S32;
#pragma unroll
    for (int ks = 0; ks < KC32 / 4; ++ks) {
      const int kk = 4 * ks + kq;
      float a[4], b[2];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = As[(64 * wr + 16 * i + l16) * S32 + kk];
#pragma unroll
      for (int c = 0; c < 2; ++c) b[c] = Bs[(32 * wc + 16 * c + l16) * S32 + kk];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int c = 0; c < 2; ++c)
          acc[i][c] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], b[c], acc[i][c], 0, 0, 0);
    }
    if (st + 1 < nst) sstore(cur ^ 1);
    __syncthreads();
  }
  store_lowp<TOUT>(C, ldc, M, N, lower_only, acc);
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

__device__ __forceinline__ void run_unit(const TaskDesc &d, int unit, double *lds) {
  int p, q;
  bool lower_only;
  int M, N;
  if (d.kind == K_SYRK) {
    p = 0;
    while ((p + 1) * (p + 2) / 2 <= unit) ++p;
    q = unit - p * (p + 1) / 2;
    M = min(GEMM_UNIT, d.m - p * GEMM_UNIT);
    N = min(GEMM_UNIT, d.m - q * GEMM_UNIT);
    lower_only = p == q;
  } else {
    const int qn = (d.n + GEMM_UNIT - 1) / GEMM_UNIT;
    p = unit / qn;
    q = unit % qn;
    M = min(GEMM_UNIT, d.m - p * GEMM_UNIT);
    N = min(GEMM_UNIT, d.n - q * GEMM_UNIT);
    lower_only = false;
  }
  const int r0 = p * GEMM_UNIT, c0 = q * GEMM_UNIT;
  // SYRK reads both operands from its one input
  const void *bsrc = d.kind == K_SYRK ? d.a : d.b;
  const int64_t ldb = d.kind == K_SYRK ? d.lda : d.ldb;
  const int64_t coff = (int64_t)r0 * d.ldc + c0;
  if (d.ta == T_F64) {
    block_f64((gdouble *)d.c + coff, d.ldc, (const gdouble *)d.a + (int64_t)r0 * d.lda, d.lda,
              (const gdouble *)bsrc + (int64_t)c0 * ldb, ldb, M, N, d.k, lower_only, lds);
  } else if (d.ta == T_F32) {
    const gfloat *A = (const gfloat *)d.a + (int64_t)r0 * d.lda;
    const gfloat *B = (const gfloat *)bsrc + (int64_t)c0 * ldb;
    if (d.tc == T_F64)
      block_f32<double>((gdouble *)d.c + coff, d.ldc, A, d.lda, B, ldb, M, N, d.k, lower_only,
                         (float *)lds);
    else
      block_f32<float>((gfloat *)d.c + coff, d.ldc, A, d.lda, B, ldb, M, N, d.k, lower_only,
                        (float *)lds);
  } else {
    const gbf16 *A = (const gbf16 *)d.a + (int64_t)r0 * d.lda;
    const gbf16 *B = (const gbf16 *)bsrc + (int64_t)c0 * ldb;
    if (d.tc == T_F64)
      block_bf16<double>((gdouble *)d.c + coff, d.ldc, A, d.lda, B, ldb, M, N, d.k, lower_only,
                          (__bf16 *)lds);
    else
      block_bf16<float>((gfloat *)d.c + coff, d.ldc, A, d.lda, B, ldb, M, N, d.k, lower_only,
                         (__bf16 *)lds);
  }
}

__device__ __forceinline__ uint64_t uniform_u64(uint64_t v) {
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
  return ((uint64_t)hi << 32) | lo;
}

__global__ void __launch_bounds__(GT, 1) dc_gemm_kernel(LevelArgs A) {
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
    if (!__builtin_amdgcn_readfirstlane(s_skip)) run_unit(d, u, lds);
    if (A.trace && tid == 0) {
      atomicMax((unsigned long long *)&A.trace[3 * t + 1], (unsigned long long)wall_clock64());
      A.trace[3 * t + 2] = blockIdx.x;
    }
    __syncthreads();
  }
}

constexpr int GEMM_KERNEL_LDS = 2 * STAGE64 * (int)sizeof(double);
static_assert(2 * STAGE32 * (int)sizeof(float) <= GEMM_KERNEL_LDS, "f32 lds");
static_assert(2 * STAGE16 * 2 <= GEMM_KERNEL_LDS, "bf16 lds");

}  // namespace

int dcx_launch_gemm(const LevelArgs &args, int workers, void *stream) {
  hipLaunchKernelGGL(dc_gemm_kernel, dim3(workers), dim3(GT), GEMM_KERNEL_LDS, (hipStream_t)stream,
                     args);
  return (int)hipGetLastError();
}

int dcx_gemm_setup(void) {
  return (int)hipFuncSetAttribute((const void *)dc_gemm_kernel,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, GEMM_KERNEL_LDS);
}

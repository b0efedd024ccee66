// Internal ABI between the host runtime and the device executor.
// Not part of the public interface (include/dagchol.h).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "queue.h"

namespace dcx {

// Task kinds: the same numbering as dc_kind in the public header.
enum Kind : int32_t {
  K_POTRF = 0, K_TRSM = 1, K_SYRK = 2, K_GEMM = 3,
  K_TRSM_L = 4, K_GEMM_RHS_N = 5, K_TRSM_LT = 6, K_GEMM_RHS_T = 7,
  K_SCAL = 8, K_CAST = 9, K_RESID = 10, K_AXPY = 11, K_TRSM_CAST = 12,
  K_TRTRI = 13, K_TRSM_INV = 14, K_TRSM_INV_CAST = 15, K_TRSM_L_INV = 16, K_TRSM_LT_INV = 17,
  K_NUM = 18
};

enum DType : int32_t { T_F64 = 0, T_F32 = 1, T_BF16 = 2 };

// Output sub-block edge of one GEMM/SYRK work unit.
constexpr int GEMM_UNIT = 128;
// Rows of the solve/residual/cast work units.
constexpr int ROW_UNIT = 64;
// Column block of POTRF and TRSM.
constexpr int PANEL = 16;
// Largest tile edge the POTRF and TRSM units accept.
constexpr int MAX_TILE = 512;
// Rows of X one TRSM unit keeps in LDS.
constexpr int TRSM_ROWS = 16;

__host__ __device__ inline int trsm_rows(int) { return TRSM_ROWS; }

// Padded LDS row stride (doubles) for panels of up to nb columns: a
// multiple of 32 plus 2, so that 16 consecutive rows read at one column
// fall in distinct bank pairs.
__host__ __device__ inline int panel_stride(int nb) { return (nb + 31) / 32 * 32 + 2; }

// LDS (doubles) each panel-kernel unit kind needs; the largest bounds the
// panel kernel's dynamic LDS.
__host__ __device__ inline int trsm_lds_doubles(int nb) {
  // X rows and L rows (16 x panel stride each), the transposed diagonal
  // block (16 x 18) and its 16 reciprocal pivots
  return 2 * TRSM_ROWS * panel_stride(nb) + PANEL * (PANEL + 2) + PANEL;
}
// Largest tile order the register-resident POTRF takes (every 16x16 block
// of its lower triangle held in MFMA accumulators across the four waves).
constexpr int RPOTRF_MAX = 256;
__host__ __device__ inline int potrf_lds_doubles(int nb) {
  // above RPOTRF_MAX the left-looking POTRFs, with the pivot rows left of
  // the panel (16 x panel stride) and either the published pivot rows (16 x
  // 17, the full instance's) or the transposed diagonal block (16 x 18) and
  // its 16 reciprocal pivots (the instance of its own), and a flag; up to
  // RPOTRF_MAX the larger of that and the register-resident one, with two
  // panel buffers of nb (rounded to 16) rows of 17 doubles, the transposed
  // pivot block, its reciprocal pivots and a flag
  const int left = PANEL * panel_stride(nb) + PANEL * (PANEL + 2) + PANEL + 8;
  const int regs = 2 * ((nb + 15) / 16 * 16) * (PANEL + 1) + PANEL * (PANEL + 2) + PANEL + 8;
  return nb <= RPOTRF_MAX && regs > left ? regs : left;
}
// Solve units (TRSM_L, TRSM_LT): the right-hand-side columns of the tile
// (nb x 16, row stride BSS: 16 lanes reading one column of 16 different rows
// hit distinct banks), partial sums [16 rows][16 slices][16 cols], their
// reduction [16][16] and the 16x16 diagonal block of L.
constexpr int BSS = 17;
__host__ __device__ constexpr int solve_lds_doubles(int nb) {
  return (nb + 15) / 16 * 16 * BSS + 16 * 16 * 16 + 16 * 16 + 16 * 17;
}
// Rows of D one unit of an out-of-place diagonal solve step (TRSM_L_INV,
// TRSM_LT_INV) produces.
constexpr int SOLVE_INV_ROWS = 16;
// Rows of a right-hand-side update unit (GEMM_RHS_N, GEMM_RHS_T) and its LDS.
constexpr int RHS_ROWS = 16;
// instances of the level kernel
constexpr int LI_FULL = 0, LI_LIGHT = 1, LI_RHS = 2, LI_POTRF = 3, LI_POTRF_LL = 4;
constexpr int RHS_LDS_DOUBLES = 16 * 16 * 8;
constexpr int PANEL_LDS_DOUBLES = 2 * TRSM_ROWS * (MAX_TILE + 2) + PANEL * (PANEL + 2) + PANEL;

// One task, as the executor reads it (128 bytes).
struct TaskDesc {
  int32_t kind;
  int32_t nunits;
  int32_t m, n, k;        // extents (meaning per kind, see device.hip)
  int32_t ta, tb, tc;     // dtypes of buffers a, b, c
  int32_t matrix;         // numerical-status slot, -1 if none
  int32_t flags;
  int64_t lda, ldb, ldc, ldd;
  void *a, *b, *c, *d;
  int64_t row0;           // global row offset of a POTRF tile
  double alpha;           // scalar argument
  int64_t pad0;
};
static_assert(sizeof(TaskDesc) == 128, "descriptor size");

constexpr int MAX_LANES = 4;

// Device-side view of one level launch.
struct LevelArgs {
  const TaskDesc *desc;
  const uint64_t *items;   // (task << 32 | unit), levels concatenated
  int64_t begin;           // first item of this level
  int64_t count;           // items in this level
  unsigned long long *counter;  // next item to take (zero before the launch)
  int32_t *failed;         // per matrix: nonzero after a breakdown
  int64_t *info;           // per matrix: 0 or 1-based breakdown column
  int64_t *trace;          // optional: per task start, end (clock ticks), worker
};

// Device-side view of one ready-queue executor launch: the graph's
// descriptors and queue state (queue.h), the worker class this launch
// serves, the per-matrix status words and the optional trace.
struct QueueArgs {
  const TaskDesc *desc;
  dcq::View q;
  int32_t cls;
  int32_t *failed;
  int64_t *info;
  int64_t *trace;
};

}  // namespace dcx

// Launches one level on `stream` (a hipStream_t); returns a hipError_t value.
// inst: the instance of the level kernel (dcx::LI_FULL for any units but
// POTRF, LI_LIGHT for residual and elementwise units only, LI_RHS for solve
// right-hand-side updates only, LI_POTRF for POTRF units of order up to
// RPOTRF_MAX only, LI_POTRF_LL for larger POTRF units only).
extern "C++" int dcx_launch_level(const dcx::LevelArgs &args, int workers, size_t lds_bytes,
                                  int inst, void *stream);
// Allows the level kernel its largest dynamic LDS size.
extern "C++" int dcx_level_setup(void);
// Launches the GEMM/SYRK kernel for inputs of dtype ta (T_F64 or T_F32) of
// one level on `stream` (work items are pairs of units).
extern "C++" int dcx_launch_gemm(const dcx::LevelArgs &args, int workers, int ta, void *stream);
// Launches the GEMM/SYRK kernel for BF16 inputs of one level on `stream`.
extern "C++" int dcx_launch_gemm_lowp(const dcx::LevelArgs &args, int workers, void *stream);
// Allows the GEMM/SYRK kernels their dynamic LDS sizes.
extern "C++" int dcx_gemm_setup(void);
// Launches the ready-queue workers of the panel class (instance inst) on
// `stream`.
extern "C++" int dcx_launch_queue_panel(const dcx::QueueArgs &args, int workers,
                                        size_t lds_bytes, int inst, void *stream);
// Launches the ready-queue workers of a GEMM class (dcq::CL_G64, CL_G32 or
// CL_LOWP, args.cls) on `stream`.
extern "C++" int dcx_launch_queue_gemm(const dcx::QueueArgs &args, int workers, void *stream);
// The fixed scratch of the calls that allocate nothing: looks up the device
// address of the scratch array on `device` (current) once; returns a
// hipError_t value.
extern "C++" int dcx_noalloc_setup(int device);
// The scratch array's device address on `device`, the host staging area and
// their size; 0, or -1 before dcx_noalloc_setup succeeded on that device.
extern "C++" int dcx_noalloc_scratch(int device, void **dev, void **host, int64_t *bytes);
// Workgroups per CU the queue panel kernel (instance inst) keeps resident
// with lds_bytes of LDS.
extern "C++" int dcx_queue_occupancy(size_t lds_bytes, int inst, int *blocks_per_cu);
// Workgroups per CU the level kernel keeps resident with lds_bytes of LDS.
extern "C++" int dcx_level_occupancy(size_t lds_bytes, int inst, int *blocks_per_cu);

// Shared device/host definitions of the HIP R-matrix library (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#include "hprmat.h"

namespace hp {

// ---------------------------------------------------------------- complex --
template <typename T>
struct cplx {
  T re, im;
};

template <typename T>
__host__ __device__ __forceinline__ cplx<T> cmk(T re, T im) { return cplx<T>{re, im}; }
template <typename T>
__host__ __device__ __forceinline__ cplx<T> cadd(cplx<T> a, cplx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <typename T>
__host__ __device__ __forceinline__ cplx<T> csub(cplx<T> a, cplx<T> b) { return {a.re - b.re, a.im - b.im}; }
template <typename T>
__host__ __device__ __forceinline__ cplx<T> cmul(cplx<T> a, cplx<T> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
// a - b*c (the elimination update)
template <typename T>
__host__ __device__ __forceinline__ cplx<T> cfms(cplx<T> a, cplx<T> b, cplx<T> c) {
  return {a.re - (b.re * c.re - b.im * c.im), a.im - (b.re * c.im + b.im * c.re)};
}
template <typename T>
__host__ __device__ __forceinline__ T cabs1(cplx<T> a) {
  return (a.re < 0 ? -a.re : a.re) + (a.im < 0 ? -a.im : a.im);
}
// 1 / z with scaling against overflow (Smith's method)
template <typename T>
__host__ __device__ __forceinline__ cplx<T> crcp(cplx<T> z) {
  T ar = z.re < 0 ? -z.re : z.re, ai = z.im < 0 ? -z.im : z.im;
  if (ar >= ai) {
    T t = z.im / z.re, d = z.re + z.im * t;
    return {T(1) / d, -t / d};
  } else {
    T t = z.re / z.im, d = z.re * t + z.im;
    return {t / d, T(-1) / d};
  }
}
template <typename T>
__host__ __device__ __forceinline__ cplx<T> cdiv(cplx<T> a, cplx<T> b) { return cmul(a, crcp(b)); }

// --------------------------------------------------------------- tracing --
enum TraceCat {
  TR_ASSEMBLE = 0, TR_PANEL, TR_LASWP, TR_TRSM, TR_GEMM64, TR_GEMM32, TR_RESIDUAL, TR_REFINE, TR_RMATRIX,
  TR_SMATRIX, TR_GEMM16, TR_COUNT
};
static_assert(TR_COUNT == HP_TRACE_STAGES, "trace stage count");
bool trace_on();
// Brackets the launches issued during its lifetime with events on `st`.
class TraceScope {
 public:
  TraceScope(int cat, hipStream_t st, double flops, double bytes);
  ~TraceScope();
  TraceScope(const TraceScope &) = delete;
  TraceScope &operator=(const TraceScope &) = delete;

 private:
  int cat_;
  hipStream_t st_;
  double flops_, bytes_;
  void *a_;
};

// ------------------------------------------------------------ constants --
constexpr int kPanelWidth = 32;     // columns factored by one cooperative panel launch
constexpr int kOuterBlock = 256;    // columns per trailing-update step (GEMM K)
constexpr int kInvBlock = 128;      // rows of an inverted diagonal block of an FP32 factor
// Default convergence threshold of the FP64 refinement of FP32 factors on the
// relative correction c = max_c |d_c| / |x_c|.  Each step contracts the error
// by rho ~ kappa u32, and c estimates the error before the step, so the error
// left after applying a correction c is ~ rho c <= kappa u32 c; once
// c <= u64 / u32 = 2^-53 / 2^-24 it is below kappa u64, the accuracy of a
// backward-stable FP64 solve.  Further steps only move the iterate within
// that floor.
constexpr double kRefineTol = 0x1p-29;
// A correction that stops shrinking (more than half the previous one) means
// the iterate sits at the accuracy an FP64 residual resolves.  That floor is
// about kappa u64, and refinement of FP32 factors contracts only while
// kappa u32 < 1, i.e. while kappa u64 < u64 / u32 = 2^-29.  A stall is
// therefore accepted as converged only if the stalled correction itself is
// within a factor 8 of that bound; a stall above it means the factor does not
// contract (the ill-conditioned case of the paper's Fig. illcond) and is
// reported as non-convergence, which sends the caller to the FP64 solve.
constexpr double kStallTol = 0x1p-26;
constexpr int kMaxPanelGroups = 256;  // workgroups of one cooperative panel grid (at most one per CU)
constexpr unsigned kSpinLimit = 1u << 22;  // bounded grid-barrier wait (a few seconds)

inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Workspace carve-up shared by all entry points (offsets in bytes).
struct Workspace {
  size_t sync_off, sync_bytes;      // grid-barrier counters
  size_t slot_off, slot_bytes;      // panel pivot-candidate slots
  size_t flag_off;                  // device status flags
  size_t rhs_off, rhs_bytes;        // working-precision right-hand sides (n x nrhs)
  size_t res_off, res_bytes;        // FP64 residual (n x nrhs)
  size_t aux_off, aux_bytes;        // nrhs x nrhs complex128 (collision-matrix solve)
  size_t red_off, red_bytes;        // reductions, Coulomb values, small index arrays
  size_t inv_off, inv_bytes;        // inverted diagonal blocks of an FP32 factor
  // FP32 solves with nrhs > 0 only: the transformed L, its 256-row
  // diagonal-block inverses, a second n x nrhs buffer and build scratch
  size_t wv_off, wv_bytes, inv2_off, inv2_bytes, z_off, z_bytes, wtmp_off, wtmp_bytes;
  // FP32 factorizations: one 128-row half of the U12 block row (128 x n)
  size_t u12_off, u12_bytes;
  // HP_C64H factorizations: the split-FP16 operands of the trailing update
  // (L21 rows and U12 columns with their scales)
  bool h3;
  size_t h3a_off, h3b_off, h3_bytes;
  size_t total;
};
// Storage precision of the factors: HP_C64H factors are complex FP32 like HP_C64.
inline bool is_c64(int prec) { return prec == HP_C64 || prec == HP_C64H; }
inline bool prec_ok(int prec) { return prec == HP_C128 || prec == HP_C64 || prec == HP_C64H; }
Workspace plan_workspace(int n, int nrhs, int prec);

// Internal launchers (defined in lu.hip).
template <typename T>
int lu_factor(int n, cplx<T> *A, long lda, int *ipiv, int *perm, int *info, char *work,
              const Workspace &ws, hipStream_t st);
// `inv`: room for the inverted diagonal blocks (FP32 factors; nullptr selects
// substitution, the only FP64 mode).
template <typename T>
int lu_solve(int n, int nrhs, const cplx<T> *LU, long lda, const int *perm, cplx<T> *X, long ldx,
             cplx<T> *tmp, cplx<T> *inv, hipStream_t st);
template <typename T>
int lu_solve_permuted(int n, int nrhs, const cplx<T> *LU, long lda, cplx<T> *Y, long ldy, const cplx<T> *inv,
                      hipStream_t st);
// The backward half of lu_solve_permuted: Y <- U^-1 Y in place.
template <typename T>
int lu_solve_upper(int n, int nrhs, const cplx<T> *LU, long lda, cplx<T> *Y, long ldy, const cplx<T> *inv,
                   hipStream_t st);
// Inverts the diagonal blocks of an FP32 factor into `inv` (inverse_bytes(n, HP_C64) bytes).
template <typename T>
int solve_inverses(int n, const cplx<T> *LU, long lda, cplx<T> *inv, hipStream_t st);
size_t inverse_bytes(int n, int prec);
template <typename T>
int gemm_sub(int M, int N, int K, const cplx<T> *A, long lda, const cplx<T> *B, long ldb, cplx<T> *C,
             long ldc, hipStream_t st);
// batched: matrix b of A, B, C starts at A + b*sa, B + b*sb, C + b*sc
template <typename T>
int gemm_sub_batched(int M, int N, int K, const cplx<T> *A, long lda, long sa, const cplx<T> *B, long ldb,
                     long sb, cplx<T> *C, long ldc, long sc, int batch, hipStream_t st);
// batched C = alpha A B (C is written, never read; it must not overlap A or B)
template <typename T>
int gemm_set_batched(int M, int N, int K, T alpha, const cplx<T> *A, long lda, long sa, const cplx<T> *B, long ldb,
                     long sb, cplx<T> *C, long ldc, long sc, int batch, hipStream_t st);
size_t factor_sync_bytes(int n);
// Split-FP16 trailing update (gemm_h3.hip): operand conversion and product.
size_t h3_operand_bytes(int rows, int K);
int h3_convert_rows(int M, int K, const cplx<float> *L, long lda, void *buf, hipStream_t st);
int h3_convert_cols(int N, int K, const cplx<float> *U, long ldb, void *buf, hipStream_t st);
int gemm_h3_sub(int M, int N, int K, const void *abuf, int Mtot, int r0, const void *bbuf, int Ntot, int c0,
                cplx<float> *C, long ldc, hipStream_t st);
size_t factor_slot_bytes();
// Transformed form of an FP32 factor for repeated solves (wsolve.hip)
size_t wform_bytes(int n);
size_t wform_inv_bytes(int n);
size_t wform_tmp_bytes(int n);
int wform_build(int n, const cplx<float> *LU, long lda, const cplx<float> *inv, cplx<float> *inv2, cplx<float> *tmp,
                cplx<float> *W, hipStream_t st);
int wform_solve(int n, int nrhs, const cplx<float> *LU, long lda, const cplx<float> *inv, const cplx<float> *W,
                const cplx<float> *inv2, cplx<float> *Y, long ldy, cplx<float> *Z, long ldz, hipStream_t st);


// Direct global -> LDS load (global_load_lds_dwordx4) of one 16-byte chunk per
// lane: a wavefront's 64 chunks land in 64 consecutive 16-byte LDS slots from
// lds_byte_addr (uniform over the wavefront; passed in M0, which is declared
// clobbered, so the compiler keeps nothing of its own there).  Issued from
// inline assembly so the compiler neither reorders it nor waits for it; a
// thread waits for its own loads with wait_vmcnt before the barrier that
// publishes them.
__device__ __forceinline__ void lds_direct_load16(unsigned lds_byte_addr, const void *src) {
  const unsigned m0v = __builtin_amdgcn_readfirstlane(lds_byte_addr);
  // one wait state between the M0 write and the LDS-DMA load that reads it
  asm volatile("s_mov_b32 m0, %0\n\ts_nop 0\n\tglobal_load_lds_dwordx4 %1, off" ::"s"(m0v), "v"(src)
               : "memory", "m0");
}

// s_waitcnt with vmcnt <= n (0 <= n < 64) and the other counters unconstrained
// (gfx9 encoding: vmcnt low bits [3:0], high bits [15:14], expcnt [6:4],
// lgkmcnt [11:8]).  Vector memory operations complete in issue order, so this
// waits for all but the n most recent.
template <int n>
__device__ __forceinline__ void wait_vmcnt() {
  static_assert(n >= 0 && n < 64, "vmcnt range");
  __builtin_amdgcn_s_waitcnt((n & 15) | (7 << 4) | (15 << 8) | ((n >> 4) << 14));
}

}  // namespace hp

namespace hp {
// Records the failing HIP call (file, line, HIP error text) for hp_last_error().
void note_hip_error(hipError_t e, const char *file, int line);
// Raises the dynamic-LDS limit of a kernel when a launch needs more than the
// default 64 KB (once per kernel and size).
int ensure_dynamic_lds(const void *func, size_t bytes);
}  // namespace hp

#define HP_CHECK_HIP(x)                                 \
  do {                                                  \
    hipError_t e_ = (x);                                \
    if (e_ != hipSuccess) {                             \
      hp::note_hip_error(e_, __FILE__, __LINE__);       \
      return HP_ERR_HIP;                                \
    }                                                   \
  } while (0)

#define HP_CHECK_LAUNCH() HP_CHECK_HIP(hipGetLastError())

// Trailing update of the FP32 factorization on the FP16 matrix cores: the
// optional FP16 variant of the mixed-precision solve, under row and column
// scaling (Sec. 3.2 and Sec. 3.4 run the factorization in single precision;
// here its dominant product runs in FP16 with FP32 accumulation).
//
// C -= L21 U12 with L21 (M x K) and U12 (K x N) complex FP32.  Each row m of
// L21 is scaled by a power of two r_m and each column n of U12 by c_n so
// that every real and imaginary part lies in [-1, 1] (exact: powers of two),
// and every scaled value x is split into two FP16 words x = hi + lo + e,
// hi = fp16(x), lo = fp16(x - hi), |e| <= 2^-22 |x| + 2^-25 (the low word's
// subnormal spacing).  A real product x y is formed from three FP16 matrix-
// core products hi hi' + hi lo' + lo hi' (the dropped lo lo' is below
// 2^-22 |x y|), accumulated in FP32; a complex product takes four real ones
// (Re: ArBr - AiBi, Im: ArBi + AiBr), so twelve FP16 products per complex
// product, at sixteen times the FP32 matrix-core rate.  The FP32 panel,
// block row and solves are unchanged; the FP64 refinement absorbs the
// update's rounding like that of the FP32 product.
//
// Operand layout (written by the conversion kernels): per row of L21 (per
// column of U12), K / 8 chunks of 8 consecutive k, each chunk four planes
// (re hi, re lo, im hi, im lo) of 8 FP16 = 16 bytes: the 16-byte unit an
// MFMA lane supplies (v_mfma_f32_16x16x32_f16: lane l gives row l % 16 and k
// = 8 (l / 16) + 0..7 of A, column l % 16 and the same k of B; the
// accumulator rows are 4 (l / 16) + r).
#include "common.h"

#include <cstdlib>

namespace hp {

typedef _Float16 h8 __attribute__((ext_vector_type(8)));
typedef float f4v __attribute__((ext_vector_type(4)));

constexpr int kH3BK = 32;               // k per stage (one MFMA)
constexpr int kH3BM = 64, kH3BN = 128;  // workgroup tile
constexpr int kH3Units = kH3BK / 8 * 4;  // 16-byte units per row per stage (16)

// Power-of-two scale s with max |v| / s <= 1 (1 for an all-zero vector).
__device__ __forceinline__ float pow2_scale(float m) {
  if (!(m > 0.f)) return 1.f;
  int e;
  const float f = frexpf(m, &e);  // m = f 2^e, f in [0.5, 1)
  (void)f;
  return ldexpf(1.f, e);          // m / 2^e < 1
}

__device__ __forceinline__ void split16(float x, _Float16 &hi, _Float16 &lo) {
  hi = (_Float16)x;
  lo = (_Float16)(x - (float)hi);
}

// Rows of L21 (M x K, leading dimension lda): one wavefront per row, lane q
// handles chunk q of 8 k (K <= 512); the row's scale goes to rs[m].
__global__ __launch_bounds__(256) void h3_rows_kernel(int M, int K, const cplx<float> *__restrict__ L, long lda,
                                                      h8 *__restrict__ Ah, float *__restrict__ rs) {
  const int m = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (m >= M) return;
  const int nch = K / 8;
  const cplx<float> *row = L + (long)m * lda;
  cplx<float> v[8];
  float mx = 0.f;
  if (lane < nch) {
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      v[i] = row[lane * 8 + i];
      mx = fmaxf(mx, fmaxf(fabsf(v[i].re), fabsf(v[i].im)));
    }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) mx = fmaxf(mx, __shfl_xor(mx, off));
  const float s = pow2_scale(mx), inv = 1.f / s;
  if (lane == 0) rs[m] = s;
  if (lane < nch) {
    h8 rh, rl, ih, il;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      _Float16 a, b;
      split16(v[i].re * inv, a, b);
      rh[i] = a;
      rl[i] = b;
      split16(v[i].im * inv, a, b);
      ih[i] = a;
      il[i] = b;
    }
    h8 *dst = Ah + ((long)m * nch + lane) * 4;
    dst[0] = rh;
    dst[1] = rl;
    dst[2] = ih;
    dst[3] = il;
  }
}

// Columns of U12 (K x N, leading dimension ldb): 16 columns per workgroup,
// the K x 16 tile staged in LDS (K <= 256), column maxima, then each column's
// units written contiguously.
constexpr int kH3ColTile = 16;
__global__ __launch_bounds__(256) void h3_cols_kernel(int N, int K, const cplx<float> *__restrict__ U, long ldb,
                                                      h8 *__restrict__ Bh, float *__restrict__ cs) {
  __shared__ cplx<float> tile[256][kH3ColTile + 1];
  __shared__ float smax[16][kH3ColTile];
  __shared__ float sscale[kH3ColTile];
  const int n0 = blockIdx.x * kH3ColTile;
  const int tid = threadIdx.x;
  const int c = tid & (kH3ColTile - 1), rg = tid >> 4;  // 16 row groups of 16 threads
  float mx = 0.f;
  for (int k = rg; k < K; k += 16) {
    const cplx<float> x = (n0 + c < N) ? U[(long)k * ldb + n0 + c] : cplx<float>{0.f, 0.f};
    tile[k][c] = x;
    mx = fmaxf(mx, fmaxf(fabsf(x.re), fabsf(x.im)));
  }
  smax[rg][c] = mx;
  __syncthreads();
  if (tid < kH3ColTile) {
    float m = 0.f;
#pragma unroll
    for (int q = 0; q < 16; ++q) m = fmaxf(m, smax[q][tid]);
    const float s = pow2_scale(m);
    sscale[tid] = s;
    if (n0 + tid < N) cs[n0 + tid] = s;
  }
  __syncthreads();
  // unit (column cc, chunk q): 8 consecutive k of one column, four planes
  const int nch = K / 8;
  for (int u = tid; u < kH3ColTile * nch; u += 256) {
    const int cc = u / nch, q = u - cc * nch;
    if (n0 + cc >= N) continue;
    const float inv = 1.f / sscale[cc];
    h8 rh, rl, ih, il;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const cplx<float> x = tile[q * 8 + i][cc];
      _Float16 a, b;
      split16(x.re * inv, a, b);
      rh[i] = a;
      rl[i] = b;
      split16(x.im * inv, a, b);
      ih[i] = a;
      il[i] = b;
    }
    h8 *dst = Bh + ((long)(n0 + cc) * nch + q) * 4;
    dst[0] = rh;
    dst[1] = rl;
    dst[2] = ih;
    dst[3] = il;
  }
}

// C (M x N complex FP32, ldc) -= diag(rs) (Ah Bh^T) diag(cs) with the split
// FP16 products.  Workgroup tile 64 x 128, four wavefronts of 32 x 64 (2 x 4
// MFMA tiles), K in stages of 32 through double-buffered LDS (48 KB a
// stage), filled by direct global -> LDS loads.  In LDS a row's (column's)
// 16 units of a stage sit at slot u ^ (row & 15), so that the 16 rows an
// MFMA operand read touches hit distinct banks; the permutation is applied
// on the source side of the loads.  Tiles are walked in groups of 8 row
// blocks with XCD-contiguous ranges of workgroup ids (as the FP32 kernel).
__global__ __launch_bounds__(256, 1) void gemm_h3_kernel(int M, int N, int K, const h8 *__restrict__ Ah,
                                                         const float *__restrict__ rs, const h8 *__restrict__ Bh,
                                                         const float *__restrict__ cs, cplx<float> *__restrict__ C,
                                                         long ldc, int tm, int tn, int total, int per_xcd) {
  constexpr int BM = kH3BM, BN = kH3BN, U = kH3Units;
  constexpr int ASZ = BM * U, BSZ = BN * U;      // units per stage
  constexpr int APW = ASZ / 64 / 4, BPW = BSZ / 64 / 4;  // wave-loads per wavefront per stage
  extern __shared__ __align__(16) char smem_raw[];
  h8 *As = reinterpret_cast<h8 *>(smem_raw);  // [2][BM][16]
  h8 *Bs = As + 2 * ASZ;                      // [2][BN][16]

  const int bid = blockIdx.x;
  const int t = (bid & 7) * per_xcd + (bid >> 3);
  if (t >= total) return;
  constexpr int kGroup = 8;
  const int grp = t / (kGroup * tn);
  const int first_m = grp * kGroup;
  const int gm = min(kGroup, tm - first_m);
  const int in_grp = t - grp * kGroup * tn;
  const int m0 = (first_m + in_grp % gm) * BM, n0 = (in_grp / gm) * BN;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 64;
  const int nch = K / 8;

  // source units of this lane (stage 0): wave-load q covers rows 4q .. 4q+3,
  // lane -> row 4q + lane / 16, slot lane % 16, global unit slot ^ (row & 15)
  const h8 *asrc[APW];
  const h8 *bsrc[BPW];
#pragma unroll
  for (int i = 0; i < APW; ++i) {
    const int q = wave * APW + i;
    const int row = 4 * q + (lane >> 4), slot = lane & 15;
    asrc[i] = Ah + ((long)min(m0 + row, M - 1) * nch) * 4 + (slot ^ (row & 15));
  }
#pragma unroll
  for (int i = 0; i < BPW; ++i) {
    const int q = wave * BPW + i;
    const int col = 4 * q + (lane >> 4), slot = lane & 15;
    bsrc[i] = Bh + ((long)min(n0 + col, N - 1) * nch) * 4 + (slot ^ (col & 15));
  }
  const unsigned lds0 = (unsigned)(size_t)(const __attribute__((address_space(3))) void *)As;
  auto issue = [&](int buf, int kc) {  // kc: first chunk of the stage
#pragma unroll
    for (int i = 0; i < APW; ++i)
      lds_direct_load16(lds0 + (unsigned)((buf * ASZ + (wave * APW + i) * 64) * 16), asrc[i] + (long)kc * 4);
#pragma unroll
    for (int i = 0; i < BPW; ++i)
      lds_direct_load16(lds0 + (unsigned)((2 * ASZ + buf * BSZ + (wave * BPW + i) * 64) * 16), bsrc[i] + (long)kc * 4);
  };

  f4v acc_rr[2][4], acc_ii[2][4], acc_im[2][4];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc_rr[i][j] = acc_ii[i][j] = acc_im[i][j] = f4v{0.f, 0.f, 0.f, 0.f};
  const int fr = lane & 15, g = lane >> 4;  // operand row/column in the tile, k chunk of the stage
  const int nk = K / kH3BK;
  issue(0, 0);
  for (int kt = 0; kt < nk; ++kt) {
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (kt + 1 < nk) issue((kt + 1) & 1, (kt + 1) * (kH3BK / 8));
    const h8 *as = As + (kt & 1) * ASZ;
    const h8 *bs = Bs + (kt & 1) * BSZ;
    h8 a[2][4];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const int row = wm + i * 16 + fr;
#pragma unroll
      for (int p = 0; p < 4; ++p) a[i][p] = as[row * U + ((g * 4 + p) ^ (row & 15))];
    }
    // per tile, the three products of each real product in turn (hi hi,
    // hi lo, lo hi) into one accumulator: measured on the N = 25600 system,
    // this order refines like the FP32 product (contraction 0.03 per step);
    // the same sums issued product by product across the tiles, or with the
    // hi lo and lo hi terms in accumulators of their own, contracted 0.25
    // and 0.1 per step (the matrix cores' FP32 accumulation is not
    // order-independent at this level)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int col = wn + j * 16 + fr;
      h8 b[4];
#pragma unroll
      for (int p = 0; p < 4; ++p) b[p] = bs[col * U + ((g * 4 + p) ^ (col & 15))];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        acc_rr[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_f16(a[i][0], b[0], acc_rr[i][j], 0, 0, 0);
        acc_rr[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_f16(a[i][0], b[1], acc_rr[i][j], 0, 0, 0);
        acc_rr[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_f16(a[i][1], b[0], acc_rr[i][j], 0, 0, 0);
        acc_ii[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_f16(a[i][2], b[2], acc_ii[i][j], 0, 0, 0);
        acc_ii[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_f16(a[i][2], b[3], acc_ii[i][j], 0, 0, 0);
        acc_ii[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_f16(a[i][3], b[2], acc_ii[i][j], 0, 0, 0);
        acc_im[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_f16(a[i][0], b[2], acc_im[i][j], 0, 0, 0);
        acc_im[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_f16(a[i][0], b[3], acc_im[i][j], 0, 0, 0);
        acc_im[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_f16(a[i][1], b[2], acc_im[i][j], 0, 0, 0);
        acc_im[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_f16(a[i][2], b[0], acc_im[i][j], 0, 0, 0);
        acc_im[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_f16(a[i][2], b[1], acc_im[i][j], 0, 0, 0);
        acc_im[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_f16(a[i][3], b[0], acc_im[i][j], 0, 0, 0);
      }
    }
  }
  // epilogue: C -= r_m c_n (P_rr - P_ii, P_im), one 16-row tile at a time
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    float rsv[4];
    cplx<float> cv[4][4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int gr = min(m0 + wm + i * 16 + 4 * g + r, M - 1);
      rsv[r] = rs[gr];
#pragma unroll
      for (int j = 0; j < 4; ++j) cv[r][j] = C[(long)gr * ldc + min(n0 + wn + j * 16 + fr, N - 1)];
    }
    float csv[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) csv[j] = cs[min(n0 + wn + j * 16 + fr, N - 1)];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int gr = m0 + wm + i * 16 + 4 * g + r;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int gc = n0 + wn + j * 16 + fr;
        const float s = rsv[r] * csv[j];
        cplx<float> c = cv[r][j];
        c.re -= s * (acc_rr[i][j][r] - acc_ii[i][j][r]);
        c.im -= s * acc_im[i][j][r];
        if (gr < M && gc < N) C[(long)gr * ldc + gc] = c;
      }
    }
  }
}

size_t h3_operand_bytes(int rows, int K) { return align_up((size_t)rows * K * 8, 256) + align_up(sizeof(float) * (size_t)rows, 256); }

int h3_convert_rows(int M, int K, const cplx<float> *L, long lda, void *buf, hipStream_t st) {
  if (M <= 0) return HP_OK;
  if (K % kH3BK != 0 || K > 512) return HP_ERR_UNSUPPORTED;
  h8 *Ah = (h8 *)buf;
  float *rs = (float *)((char *)buf + align_up((size_t)M * K * 8, 256));
  hipLaunchKernelGGL(h3_rows_kernel, dim3((unsigned)((M + 3) / 4)), dim3(256), 0, st, M, K, L, lda, Ah, rs);
  HP_CHECK_LAUNCH();
  return HP_OK;
}

int h3_convert_cols(int N, int K, const cplx<float> *U, long ldb, void *buf, hipStream_t st) {
  if (N <= 0) return HP_OK;
  if (K % kH3BK != 0 || K > 256) return HP_ERR_UNSUPPORTED;
  h8 *Bh = (h8 *)buf;
  float *cs = (float *)((char *)buf + align_up((size_t)N * K * 8, 256));
  hipLaunchKernelGGL(h3_cols_kernel, dim3((unsigned)((N + kH3ColTile - 1) / kH3ColTile)), dim3(256), 0, st, N, K, U,
                     ldb, Bh, cs);
  HP_CHECK_LAUNCH();
  return HP_OK;
}

// C (M x N, ldc) -= (rows [r0, r0 + M) of the converted L21) (columns [c0, c0 + N)
// of the converted U12); abuf / bbuf as written by h3_convert_rows / _cols for
// Mtot rows and Ntot columns.
int gemm_h3_sub(int M, int N, int K, const void *abuf, int Mtot, int r0, const void *bbuf, int Ntot, int c0,
                cplx<float> *C, long ldc, hipStream_t st) {
  if (M <= 0 || N <= 0 || K <= 0) return HP_OK;
  if (K % kH3BK != 0 || r0 < 0 || c0 < 0 || r0 + M > Mtot || c0 + N > Ntot) return HP_ERR_ARG;
  const h8 *Ah = (const h8 *)abuf + (size_t)r0 * (K / 8) * 4;
  const float *rs = (const float *)((const char *)abuf + align_up((size_t)Mtot * K * 8, 256)) + r0;
  const h8 *Bh = (const h8 *)bbuf + (size_t)c0 * (K / 8) * 4;
  const float *cs = (const float *)((const char *)bbuf + align_up((size_t)Ntot * K * 8, 256)) + c0;
  const int tm = (M + kH3BM - 1) / kH3BM, tn = (N + kH3BN - 1) / kH3BN;
  const long total_l = (long)tm * tn;
  if (total_l > (1L << 30)) return HP_ERR_UNSUPPORTED;
  const int total = (int)total_l, per_xcd = (total + 7) / 8;
  const size_t shm = (size_t)2 * (kH3BM + kH3BN) * kH3Units * 16;
  int rc = ensure_dynamic_lds((const void *)gemm_h3_kernel, shm);
  if (rc) return rc;
  // 12 FP16 matrix-core products of 2 x 16 x 16 x 32 flops per complex 16 x 16 x 32 block
  TraceScope ts(TR_GEMM16, st, 12.0 * 2.0 * M * (double)N * K, 8.0 * 2.0 * M * (double)N);
  hipLaunchKernelGGL(gemm_h3_kernel, dim3((unsigned)(8 * per_xcd)), dim3(256), shm, st, M, N, K, Ah, rs, Bh, cs, C,
                     ldc, tm, tn, total, per_xcd);
  HP_CHECK_LAUNCH();
  return HP_OK;
}

}  // namespace hp

using namespace hp;

extern "C" int hp_gemm_h3_sub(int M, int N, int K, const void *A, long lda, const void *B, long ldb, void *C, long ldc,
                              void *work, size_t work_bytes, void *stream) {
  if (M < 0 || N < 0 || K < 0) return HP_ERR_ARG;
  if (M == 0 || N == 0 || K == 0) return HP_OK;
  if (!A || !B || !C || !work || lda < K || ldb < N || ldc < N) return HP_ERR_ARG;
  if (K % kH3BK != 0 || K > 256) return HP_ERR_UNSUPPORTED;
  const size_t ab = h3_operand_bytes(M, K), bb = h3_operand_bytes(N, K);
  if (work_bytes < ab + bb) return HP_ERR_WORKSPACE;
  hipStream_t st = (hipStream_t)stream;
  char *w = (char *)work;
  int rc;
  if ((rc = h3_convert_rows(M, K, (const cplx<float> *)A, lda, w, st))) return rc;
  if ((rc = h3_convert_cols(N, K, (const cplx<float> *)B, ldb, w + ab, st))) return rc;
  return gemm_h3_sub(M, N, K, w, M, 0, w + ab, N, 0, (cplx<float> *)C, ldc, st);
}

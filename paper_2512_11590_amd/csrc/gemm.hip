// Complex GEMM C -= A B on the matrix cores (the trailing update of the LU,
// Sec. 3.1 / 3.4, and every block update of the triangular solves).
//
// Row-major interleaved complex operands.  FP64 forms each complex product
// from four real MFMA products ("4M"):  Cr += Ar Br - Ai Bi,
// Ci += Ar Bi + Ai Br  (v_mfma_f64_16x16x4f64).  FP32 uses three ("3M"):
// P1 = Ar Br, P2 = Ai Bi, P3 = (Ar + Ai)(Br + Bi), then Cr += P1 - P2,
// Ci += P3 - P1 - P2  (v_mfma_f32_16x16x4f32): a quarter fewer matrix-core
// cycles, with the imaginary part's rounding error bounded by |A||B| instead
// of its own terms -- the FP32 factors feed the FP64 refinement, which
// absorbs that; the FP64 factorization keeps the 4M product.
//
// Tiling for CDNA4: 256 threads = 4 wavefronts in a 2 x 2 grid; a wavefront
// owns WTM x WTN MFMA tiles of 16 x 16 complex outputs.  K advances in stages
// of 16 complex staged through double-buffered LDS (A stored k-major so both
// operands read 16 consecutive complex per k), the next stage's global loads
// (16-byte vectors when the operands allow it) in flight during the MFMAs of
// the current one, one barrier per stage.  Workgroups walk the output tiles
// in groups of 8 row-blocks (column-major inside a group) so a group's A rows
// and B columns stay in one XCD's L2, and consecutive workgroup ids, which
// the hardware deals round-robin over the 8 XCDs, are remapped so that each
// XCD gets a contiguous range of tiles.
#include "common.h"

namespace hp {

template <typename T>
struct Mfma;
template <>
struct Mfma<double> {
  typedef double v4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ v4 mac(double a, double b, v4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
};
template <>
struct Mfma<float> {
  typedef float v4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ v4 mac(float a, float b, v4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
};

// Lane layout of the 16x16x4 MFMA: lane l supplies A[l%16][l/16] and
// B[l/16][l%16]; accumulator element r of lane l is D[d_row(l,r)][l%16].
// Read off the hardware with one-hot operands: the FP32 instruction returns
// rows 4*(l/16)+r, the FP64 one rows 4*r + l/16.
template <typename T>
struct MfmaLayout {
  static __device__ __forceinline__ int d_row(int l, int r) { return 4 * (l >> 4) + r; }
};
template <>
struct MfmaLayout<double> {
  static __device__ __forceinline__ int d_row(int l, int r) { return 4 * r + (l >> 4); }
};

template <typename T>
struct alignas(16) Vec16 {
  cplx<T> v[16 / sizeof(cplx<T>)];
};

template <typename T, int WTM, int WTN>
struct GemmCfg {
  static constexpr int BM = 32 * WTM;
  static constexpr int BN = 32 * WTN;
  static constexpr int BK = 16;
  static constexpr int EV = 16 / (int)sizeof(cplx<T>);         // complex per 16-byte vector
  // LDS row padding (complex): one element on the k-major A rows spreads the
  // transposing stores over banks; the B rows stay 16-byte aligned for vector
  // stores (FP32: 33 KB per workgroup, so three fit beside a panel workgroup)
  static constexpr int PADA = 1, PADB = sizeof(T) == 4 ? 0 : 1;
  static constexpr int PA = BM + PADA, PB = BN + PADB;
  static constexpr int NVA = BM * BK / EV / 256;               // A vectors per thread per stage
  static constexpr int NVB = BK * BN / EV / 256;               // B vectors per thread per stage
  static constexpr size_t lds_bytes = (size_t)2 * BK * (PA + PB) * sizeof(cplx<T>);
  static_assert(NVA >= 1 && NVB >= 1, "tile too small for 256 threads");
};

constexpr int kGroupM = 8;

// SET = false: C -= A B.  SET = true: C = alpha A B (C is not read).
template <typename T, int WTM, int WTN, bool VEC, bool SET>
__global__ __launch_bounds__(256) void gemm_sub_kernel(int M, int N, int K, const cplx<T> *__restrict__ A, long lda,
                                                       long sa, const cplx<T> *__restrict__ B, long ldb, long sb,
                                                       cplx<T> *__restrict__ C, long ldc, long sc, int tm, int tn,
                                                       int total, int per_xcd, T alpha) {
  typedef GemmCfg<T, WTM, WTN> G;
  typedef typename Mfma<T>::v4 v4;
  constexpr int BM = G::BM, BN = G::BN, BK = G::BK, EV = G::EV, PA = G::PA, PB = G::PB;
  extern __shared__ __align__(16) char smem_raw[];
  cplx<T> *As = reinterpret_cast<cplx<T> *>(smem_raw);  // [2][BK][PA]
  cplx<T> *Bs = As + 2 * BK * PA;                       // [2][BK][PB]

  // tile scheduling: XCD-contiguous ranges, grouped row-blocks
  const int bid = blockIdx.x;
  const int t = (bid & 7) * per_xcd + (bid >> 3);
  if (t >= total) return;
  const int per_batch = tm * tn;
  const int z = t / per_batch;
  const int tb = t - z * per_batch;
  const int grp = tb / (kGroupM * tn);
  const int first_m = grp * kGroupM;
  const int gm = min(kGroupM, tm - first_m);
  const int in_grp = tb - grp * kGroupM * tn;
  const int im = first_m + in_grp % gm;
  const int in = in_grp / gm;
  const int m0 = im * BM, n0 = in * BN;
  A += sa * z;
  B += sb * z;
  C += sc * z;

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = (wave >> 1) * (16 * WTM), wn = (wave & 1) * (16 * WTN);

  Vec16<T> ra[G::NVA], rb[G::NVB];
  auto load_stage = [&](int k0) {
#pragma unroll
    for (int q = 0; q < G::NVA; ++q) {
      const int v = tid + 256 * q;
      const int row = v / (BK / EV), kv = v % (BK / EV);
      const int gr = m0 + row, gk = k0 + kv * EV;
      const cplx<T> *p = A + (long)gr * lda + gk;
      if (VEC && gr < M && gk + EV <= K) {
        ra[q] = *reinterpret_cast<const Vec16<T> *>(p);
      } else {
#pragma unroll
        for (int e = 0; e < EV; ++e) {
          ra[q].v[e] = cplx<T>{T(0), T(0)};
          if (gr < M && gk + e < K) ra[q].v[e] = p[e];
        }
      }
    }
#pragma unroll
    for (int q = 0; q < G::NVB; ++q) {
      const int v = tid + 256 * q;
      const int kr = v / (BN / EV), nv = v % (BN / EV);
      const int gk = k0 + kr, gc = n0 + nv * EV;
      const cplx<T> *p = B + (long)gk * ldb + gc;
      if (VEC && gk < K && gc + EV <= N) {
        rb[q] = *reinterpret_cast<const Vec16<T> *>(p);
      } else {
#pragma unroll
        for (int e = 0; e < EV; ++e) {
          rb[q].v[e] = cplx<T>{T(0), T(0)};
          if (gk < K && gc + e < N) rb[q].v[e] = p[e];
        }
      }
    }
  };
  auto store_stage = [&](int buf) {
    cplx<T> *as = As + buf * BK * PA;
    cplx<T> *bs = Bs + buf * BK * PB;
#pragma unroll
    for (int q = 0; q < G::NVA; ++q) {
      const int v = tid + 256 * q;
      const int row = v / (BK / EV), kv = v % (BK / EV);
#pragma unroll
      for (int e = 0; e < EV; ++e) as[(kv * EV + e) * PA + row] = ra[q].v[e];
    }
#pragma unroll
    for (int q = 0; q < G::NVB; ++q) {
      const int v = tid + 256 * q;
      const int kr = v / (BN / EV), nv = v % (BN / EV);
      *reinterpret_cast<Vec16<T> *>(bs + kr * PB + nv * EV) = rb[q];
    }
  };

  // 4M: acc_re, acc_im; 3M: acc_re = P1, acc_im = P3, acc_p2 = P2
  constexpr bool M3 = sizeof(T) == 4;
  v4 acc_re[WTM][WTN], acc_im[WTM][WTN], acc_p2[WTM][WTN];
#pragma unroll
  for (int i = 0; i < WTM; ++i)
#pragma unroll
    for (int j = 0; j < WTN; ++j) {
      acc_re[i][j] = v4{0, 0, 0, 0};
      acc_im[i][j] = v4{0, 0, 0, 0};
      acc_p2[i][j] = v4{0, 0, 0, 0};
    }

  const int nk = (K + BK - 1) / BK;
  load_stage(0);
  store_stage(0);
  __syncthreads();
  const int fr = lane & 15, fk = lane >> 4;
  for (int kt = 0; kt < nk; ++kt) {
    const int cur = kt & 1;
    if (kt + 1 < nk) load_stage((kt + 1) * BK);
    const cplx<T> *as = As + cur * BK * PA;
    const cplx<T> *bs = Bs + cur * BK * PB;
#pragma unroll
    for (int ks = 0; ks < BK; ks += 4) {
      const int kk = ks + fk;
      cplx<T> af[WTM], bf[WTN];
#pragma unroll
      for (int i = 0; i < WTM; ++i) af[i] = as[kk * PA + wm + i * 16 + fr];
#pragma unroll
      for (int j = 0; j < WTN; ++j) bf[j] = bs[kk * PB + wn + j * 16 + fr];
      if constexpr (M3) {
        T bs_[WTN];
#pragma unroll
        for (int j = 0; j < WTN; ++j) bs_[j] = bf[j].re + bf[j].im;
#pragma unroll
        for (int i = 0; i < WTM; ++i) {
          const T as_ = af[i].re + af[i].im;
#pragma unroll
          for (int j = 0; j < WTN; ++j) {
            acc_re[i][j] = Mfma<T>::mac(af[i].re, bf[j].re, acc_re[i][j]);
            acc_p2[i][j] = Mfma<T>::mac(af[i].im, bf[j].im, acc_p2[i][j]);
            acc_im[i][j] = Mfma<T>::mac(as_, bs_[j], acc_im[i][j]);
          }
        }
      } else {
#pragma unroll
        for (int i = 0; i < WTM; ++i) {
          const T nai = -af[i].im;
#pragma unroll
          for (int j = 0; j < WTN; ++j) {
            acc_re[i][j] = Mfma<T>::mac(af[i].re, bf[j].re, acc_re[i][j]);
            acc_im[i][j] = Mfma<T>::mac(af[i].re, bf[j].im, acc_im[i][j]);
            acc_re[i][j] = Mfma<T>::mac(nai, bf[j].im, acc_re[i][j]);
            acc_im[i][j] = Mfma<T>::mac(af[i].im, bf[j].re, acc_im[i][j]);
          }
        }
      }
    }
    if (kt + 1 < nk) store_stage(cur ^ 1);
    __syncthreads();
  }
  // Epilogue: every C element this thread owns is loaded (at a clamped, always
  // valid address) before the first one is used, so the loads are in flight
  // together; out-of-range elements are then skipped on the store.
  cplx<T> cv[WTM][4][WTN];
#pragma unroll
  for (int i = 0; i < WTM; ++i)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int gr = min(m0 + wm + i * 16 + MfmaLayout<T>::d_row(lane, r), M - 1);
#pragma unroll
      for (int j = 0; j < WTN; ++j) {
        if constexpr (SET)
          cv[i][r][j] = cplx<T>{T(0), T(0)};
        else
          cv[i][r][j] = C[(long)gr * ldc + min(n0 + wn + j * 16 + fr, N - 1)];
      }
    }
#pragma unroll
  for (int i = 0; i < WTM; ++i)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int gr = m0 + wm + i * 16 + MfmaLayout<T>::d_row(lane, r);
#pragma unroll
      for (int j = 0; j < WTN; ++j) {
        const int gc = n0 + wn + j * 16 + fr;
        cplx<T> c = cv[i][r][j];
        if constexpr (M3) {
          const T p1 = acc_re[i][j][r], p2 = acc_p2[i][j][r], p3 = acc_im[i][j][r];
          c.re -= p1 - p2;
          c.im -= p3 - p1 - p2;
        } else {
          c.re -= acc_re[i][j][r];
          c.im -= acc_im[i][j][r];
        }
        if constexpr (SET) c = cplx<T>{-alpha * c.re, -alpha * c.im};
        if (gr < M && gc < N) C[(long)gr * ldc + gc] = c;
      }
    }
}

template <typename T, int WTM, int WTN, bool SET>
static int launch_gemm(int M, int N, int K, const cplx<T> *A, long lda, long sa, const cplx<T> *B, long ldb,
                       long sb, cplx<T> *C, long ldc, long sc, int batch, T alpha, hipStream_t st) {
  typedef GemmCfg<T, WTM, WTN> G;
  const int tm = (M + G::BM - 1) / G::BM, tn = (N + G::BN - 1) / G::BN;
  const long total_l = (long)tm * tn * batch;
  if (total_l > (1L << 30)) return HP_ERR_UNSUPPORTED;
  const int total = (int)total_l;
  const int per_xcd = (total + 7) / 8;
  // 16-byte vector loads need 16-byte aligned rows (one FP64 complex always is)
  bool vec = true;
  if (sizeof(T) == 4) {
    vec = ((uintptr_t)A % 16 == 0) && ((uintptr_t)B % 16 == 0) && (lda % 2 == 0) && (ldb % 2 == 0) &&
          (sa % 2 == 0) && (sb % 2 == 0);
  }
  const size_t shm = G::lds_bytes;
  const void *fn = vec ? (const void *)gemm_sub_kernel<T, WTM, WTN, true, SET>
                       : (const void *)gemm_sub_kernel<T, WTM, WTN, false, SET>;
  int rc = ensure_dynamic_lds(fn, shm);
  if (rc) return rc;
  dim3 grid((unsigned)(8 * per_xcd));
  if (vec)
    hipLaunchKernelGGL((gemm_sub_kernel<T, WTM, WTN, true, SET>), grid, dim3(256), shm, st, M, N, K, A, lda, sa, B,
                       ldb, sb, C, ldc, sc, tm, tn, total, per_xcd, alpha);
  else
    hipLaunchKernelGGL((gemm_sub_kernel<T, WTM, WTN, false, SET>), grid, dim3(256), shm, st, M, N, K, A, lda, sa,
                       B, ldb, sb, C, ldc, sc, tm, tn, total, per_xcd, alpha);
  HP_CHECK_LAUNCH();
  return HP_OK;
}

template <typename T>
int gemm_sub_batched(int M, int N, int K, const cplx<T> *A, long lda, long sa, const cplx<T> *B, long ldb, long sb,
                     cplx<T> *C, long ldc, long sc, int batch, hipStream_t st) {
  if (M <= 0 || N <= 0 || K <= 0 || batch <= 0) return HP_OK;
  // real matrix-core flops of the product: 8 M N K (4M, FP64) or 6 M N K (3M, FP32)
  TraceScope ts(sizeof(T) == 8 ? TR_GEMM64 : TR_GEMM32, st, (sizeof(T) == 8 ? 8.0 : 6.0) * M * (double)N * K * batch,
                2.0 * sizeof(cplx<T>) * (double)M * N * batch);
  // 64 x 64 tiles: measured on MI355X (12800^2 x 256 update, complex rate
  // 8MNK / t) at 120 TF/s in FP32 (90 TF/s of 3M matrix-core flops then, 104
  // since the epilogue loads were batched) and 57 TF/s in FP64, against
  // 79-110 TF/s and 45 TF/s for the 128-wide tiles, whose register footprint
  // leaves one wavefront per SIMD.  A variant that loads C during the last K
  // stage was 1 % faster alone but slower beside the panel (more registers).
  return launch_gemm<T, 2, 2, false>(M, N, K, A, lda, sa, B, ldb, sb, C, ldc, sc, batch, T(1), st);
}

template <typename T>
int gemm_set_batched(int M, int N, int K, T alpha, const cplx<T> *A, long lda, long sa, const cplx<T> *B, long ldb,
                     long sb, cplx<T> *C, long ldc, long sc, int batch, hipStream_t st) {
  if (M <= 0 || N <= 0 || K <= 0 || batch <= 0) return HP_OK;
  TraceScope ts(sizeof(T) == 8 ? TR_GEMM64 : TR_GEMM32, st, (sizeof(T) == 8 ? 8.0 : 6.0) * M * (double)N * K * batch,
                1.0 * sizeof(cplx<T>) * (double)M * N * batch);
  return launch_gemm<T, 2, 2, true>(M, N, K, A, lda, sa, B, ldb, sb, C, ldc, sc, batch, alpha, st);
}

template <typename T>
int gemm_sub(int M, int N, int K, const cplx<T> *A, long lda, const cplx<T> *B, long ldb, cplx<T> *C, long ldc,
             hipStream_t st) {
  return gemm_sub_batched<T>(M, N, K, A, lda, 0, B, ldb, 0, C, ldc, 0, 1, st);
}

template int gemm_sub<double>(int, int, int, const cplx<double> *, long, const cplx<double> *, long,
                              cplx<double> *, long, hipStream_t);
template int gemm_sub<float>(int, int, int, const cplx<float> *, long, const cplx<float> *, long, cplx<float> *,
                             long, hipStream_t);
template int gemm_sub_batched<double>(int, int, int, const cplx<double> *, long, long, const cplx<double> *, long,
                                      long, cplx<double> *, long, long, int, hipStream_t);
template int gemm_sub_batched<float>(int, int, int, const cplx<float> *, long, long, const cplx<float> *, long,
                                     long, cplx<float> *, long, long, int, hipStream_t);
template int gemm_set_batched<float>(int, int, int, float, const cplx<float> *, long, long, const cplx<float> *,
                                     long, long, cplx<float> *, long, long, int, hipStream_t);
template int gemm_set_batched<double>(int, int, int, double, const cplx<double> *, long, long,
                                      const cplx<double> *, long, long, cplx<double> *, long, long, int, hipStream_t);

}  // namespace hp

using namespace hp;

extern "C" int hp_gemm_sub(int M, int N, int K, int prec, const void *A, long lda, const void *B, long ldb, void *C,
                           long ldc, void *stream) {
  if (M < 0 || N < 0 || K < 0) return HP_ERR_ARG;
  if ((M && N && K) && (!A || !B || !C || lda < K || ldb < N || ldc < N)) return HP_ERR_ARG;
  hipStream_t st = (hipStream_t)stream;
  if (prec == HP_C128)
    return gemm_sub<double>(M, N, K, (const cplx<double> *)A, lda, (const cplx<double> *)B, ldb, (cplx<double> *)C,
                            ldc, st);
  if (prec == HP_C64)
    return gemm_sub<float>(M, N, K, (const cplx<float> *)A, lda, (const cplx<float> *)B, ldb, (cplx<float> *)C, ldc,
                           st);
  return HP_ERR_ARG;
}

// Batched uneven systems: many independent coupled-channel systems (one per
// (J^pi, energy) label, N = nc*nr of a few hundred to a few thousand) solved
// side by side, one workgroup per system.
//
// At these sizes one system cannot fill the device, and the full-size path's
// per-column grid barrier would make every system latency-bound.  Here a
// single workgroup owns a system for the whole factorization (no grid
// synchronisation at all), and the device is filled by running hundreds of
// systems at once; systems are taken largest first from an atomic counter,
// so the persistent grid stays balanced.
//
//   hp_batch_build    assembly of C(E) for every system (Eq. block_structure)
//   hp_batch_factor   persistent batched LU with partial pivoting (Sec. 3.1):
//                     per panel of W columns, column steps with immediate row
//                     interchanges, the panel's block row, and the trailing
//                     update as MFMA complex tiles (3M in FP32, 4M in FP64)
//   hp_batch_solve_init / hp_batch_refine_step
//                     solves for the nc surface right-hand sides, and FP64
//                     refinement of FP32 factors (Sec. 3.2) with a per-system
//                     stop rule; one refinement step is a fixed sequence of
//                     launches with no host synchronisation (capturable)
//   hp_batch_rmatrix  R for every system (Sec. 3.1 step 4)
#include "common.h"

#include <algorithm>
#include <climits>
#include <atomic>
#include <type_traits>
#include <vector>

namespace hp {

namespace {

template <typename T>
struct BMfma;
template <>
struct BMfma<double> {
  typedef double v4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ v4 mac(double a, double b, v4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  // accumulator element r of lane l is row 4 r + l / 16 of the 16 x 16 tile
  static __device__ __forceinline__ int d_row(int l, int r) { return 4 * r + (l >> 4); }
};
template <>
struct BMfma<float> {
  typedef float v4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ v4 mac(float a, float b, v4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  // accumulator element r of lane l is row 4 (l / 16) + r
  static __device__ __forceinline__ int d_row(int l, int r) { return 4 * (l >> 4) + r; }
};

constexpr int kBK = 32;       // largest K of one workgroup GEMM (panel width, solve block)
constexpr int kBLd = 64 + 1;  // LDS row stride of the staged 64-wide tiles (complex)

// LDS of one workgroup GEMM: the A and B tiles (33 KB in FP32, 67 KB in FP64)
template <typename T>
constexpr size_t tile_lds_bytes() {
  return (size_t)2 * kBK * kBLd * sizeof(cplx<T>);
}

// One 64 x 64 output tile (m0, n0) of C[M x N] -= A[M x K] B[K x N] by one
// workgroup: K in chunks of kBK, each chunk's A and B staged k-major in LDS
// (in FP32 the next chunk's loads are in flight while the current one is
// multiplied), four wavefronts of 32 x 32 outputs, MFMA 16x16x4.  FP32:
// three real products per complex product (3M), FP64: four (4M).  A, B and
// C must not overlap.  The LDS tiles are free again when it returns (its last
// barrier follows the last product).
template <typename T>
__device__ __forceinline__ void tile_gemm_sub(int m0, int n0, int M, int N, int K, const cplx<T> *__restrict__ A, long lda,
                              const cplx<T> *__restrict__ B, long ldb, cplx<T> *__restrict__ C, long ldc,
                              cplx<T> *As, cplx<T> *Bs) {
  typedef typename BMfma<T>::v4 v4;
  constexpr bool M3 = sizeof(T) == 4;
  constexpr int NS = 64 * kBK / 256;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  const int fr = lane & 15, fk = lane >> 4;
  const cplx<T> zero{T(0), T(0)};
  cplx<T> ra[NS], rb[NS];
  // a chunk's loads at clamped addresses (in bounds, no branch to wait on);
  // out-of-range values are masked to zero when stored
  auto load = [&](int kc) __attribute__((always_inline)) {
    const int kb = min(kBK, K - kc), Kp = (kb + 3) & ~3;
#pragma unroll
    for (int u = 0; u < NS; ++u) {
      const int e = tid + 256 * u;
      const int r = e / Kp, k = e - r * Kp;
      ra[u] = A[(long)min(m0 + r, M - 1) * lda + kc + min(k, kb - 1)];
      const int kr = e >> 6, c = e & 63;
      rb[u] = B[(long)(kc + min(kr, kb - 1)) * ldb + min(n0 + c, N - 1)];
    }
  };
  v4 p1[2][2], p2[2][2], p3[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) p1[i][j] = p2[i][j] = p3[i][j] = v4{0, 0, 0, 0};
  // FP32: the next chunk's loads are issued before the current chunk's
  // products; FP64 loads each chunk at its start (its registers would not
  // fit beside the accumulators of the 4M product)
  constexpr bool kPrefetch = sizeof(T) == 4;
  if constexpr (kPrefetch) load(0);
  for (int kc = 0; kc < K; kc += kBK) {
    const int kb = min(kBK, K - kc), Kp = (kb + 3) & ~3;
    if constexpr (kPrefetch) {
#pragma unroll
      for (int u = 0; u < NS; ++u) {
        const int e = tid + 256 * u;
        if (e < 64 * Kp) {
          const int r = e / Kp, k = e - r * Kp;
          As[k * kBLd + r] = (m0 + r < M && k < kb) ? ra[u] : zero;
          const int kr = e >> 6, c = e & 63;
          Bs[kr * kBLd + c] = (kr < kb && n0 + c < N) ? rb[u] : zero;
        }
      }
    } else {
      // each value stored as it arrives (no staging registers)
#pragma unroll
      for (int u = 0; u < NS; ++u) {
        const int e = tid + 256 * u;
        if (e < 64 * Kp) {
          const int r = e / Kp, k = e - r * Kp;
          const cplx<T> va = A[(long)min(m0 + r, M - 1) * lda + kc + min(k, kb - 1)];
          const int kr = e >> 6, c = e & 63;
          const cplx<T> vb = B[(long)(kc + min(kr, kb - 1)) * ldb + min(n0 + c, N - 1)];
          As[k * kBLd + r] = (m0 + r < M && k < kb) ? va : zero;
          Bs[kr * kBLd + c] = (kr < kb && n0 + c < N) ? vb : zero;
        }
      }
    }
    __syncthreads();
    if (kPrefetch && kc + kBK < K) load(kc + kBK);
    for (int ks = 0; ks < Kp; ks += 4) {
      const int kk = ks + fk;
      cplx<T> af[2], bf[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) af[i] = As[kk * kBLd + wm + i * 16 + fr];
#pragma unroll
      for (int j = 0; j < 2; ++j) bf[j] = Bs[kk * kBLd + wn + j * 16 + fr];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          if constexpr (M3) {
            // p1 = Ar Br, p2 = Ai Bi, p3 = (Ar + Ai)(Br + Bi)
            p1[i][j] = BMfma<T>::mac(af[i].re, bf[j].re, p1[i][j]);
            p2[i][j] = BMfma<T>::mac(af[i].im, bf[j].im, p2[i][j]);
            p3[i][j] = BMfma<T>::mac(af[i].re + af[i].im, bf[j].re + bf[j].im, p3[i][j]);
          } else {
            // p1 = Ar Br - Ai Bi, p3 = Ar Bi + Ai Br
            p1[i][j] = BMfma<T>::mac(af[i].re, bf[j].re, p1[i][j]);
            p1[i][j] = BMfma<T>::mac(-af[i].im, bf[j].im, p1[i][j]);
            p3[i][j] = BMfma<T>::mac(af[i].re, bf[j].im, p3[i][j]);
            p3[i][j] = BMfma<T>::mac(af[i].im, bf[j].re, p3[i][j]);
          }
        }
    }
    __syncthreads();
  }
  // C, one 16-row tile at a time: its eight loads in flight at once
  // (clamped addresses), then the updates, stored where in range
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    cplx<T> cv[4][2];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int gr = min(m0 + wm + i * 16 + BMfma<T>::d_row(lane, r), M - 1);
#pragma unroll
      for (int j = 0; j < 2; ++j) cv[r][j] = C[(long)gr * ldc + min(n0 + wn + j * 16 + fr, N - 1)];
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int gr = m0 + wm + i * 16 + BMfma<T>::d_row(lane, r);
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int gc = n0 + wn + j * 16 + fr;
        cplx<T> c = cv[r][j];
        if constexpr (M3) {
          c.re -= p1[i][j][r] - p2[i][j][r];
          c.im -= p3[i][j][r] - p1[i][j][r] - p2[i][j][r];
        } else {
          c.re -= p1[i][j][r];
          c.im -= p3[i][j][r];
        }
        if (gr < M && gc < N) C[(long)gr * ldc + gc] = c;
      }
    }
  }
}

// FP64 form of tile_gemm_sub with the operands staged by direct
// global->LDS loads in stages of 8 (two buffers, 32 KB of LDS): the next
// stage's loads are in flight during the current stage's products, with no
// register staging and no LDS store instructions.  A is row-major [64][8] in
// LDS with element k of row r at k ^ (r/2 mod 8) (the 16 rows of one MFMA
// operand read cover a 256-byte bank window once), B row-major [8][64].
// Loads past M, N or K read clamped, in-bounds addresses; A values past K are
// zeroed before their products, the other clamped values only reach outputs
// that are not stored.
__device__ __forceinline__ void tile_gemm_sub_direct64(int m0, int n0, int M, int N, int K,
                                                       const cplx<double> *__restrict__ A, long lda,
                                                       const cplx<double> *__restrict__ B, long ldb,
                                                       cplx<double> *__restrict__ C, long ldc, cplx<double> *smem) {
  typedef BMfma<double>::v4 v4;
  constexpr int BK = 8, NBUF = 2, ASZ = 64 * BK, BSZ = BK * 64;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  const int fr = lane & 15, fk = lane >> 4;
  // this lane's two A chunks and two B chunks of a stage
  const cplx<double> *arow[2], *bcol[2];
  int ak[2], bk[2];
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const int c = (wave * 2 + i) * 64 + lane;
    const int row = c >> 3, pos = c & 7;
    arow[i] = A + (long)min(m0 + row, M - 1) * lda;
    ak[i] = pos ^ ((row >> 1) & 7);
    const int kr = c >> 6, col = c & 63;
    bcol[i] = B + min(n0 + col, N - 1);
    bk[i] = kr;
  }
  const unsigned lds0 = (unsigned)(size_t)(const __attribute__((address_space(3))) void *)smem;
  auto issue = [&](int buf, int k0) {
#pragma unroll
    for (int i = 0; i < 2; ++i)
      lds_direct_load16(lds0 + (unsigned)((buf * ASZ + (wave * 2 + i) * 64) * sizeof(cplx<double>)),
                        arow[i] + min(k0 + ak[i], K - 1));
#pragma unroll
    for (int i = 0; i < 2; ++i)
      lds_direct_load16(lds0 + (unsigned)((NBUF * ASZ + buf * BSZ + (wave * 2 + i) * 64) * sizeof(cplx<double>)),
                        bcol[i] + (long)min(k0 + bk[i], K - 1) * ldb);
  };
  v4 p1[2][2], p3[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) p1[i][j] = p3[i][j] = v4{0, 0, 0, 0};
  const int nk = (K + BK - 1) / BK;
  if (nk > 0) issue(0, 0);
  for (int kt = 0; kt < nk; ++kt) {
    wait_vmcnt<0>();
    __syncthreads();
    if (kt + 1 < nk) issue((kt + 1) & 1, (kt + 1) * BK);
    const cplx<double> *as = smem + (kt & 1) * ASZ;
    const cplx<double> *bs = smem + NBUF * ASZ + (kt & 1) * BSZ;
#pragma unroll
    for (int ks = 0; ks < BK; ks += 4) {
      const int kk = ks + fk;
      const bool live = kt * BK + kk < K;
      cplx<double> af[2], bf[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        const int row = wm + i * 16 + fr;
        af[i] = as[row * BK + (kk ^ ((row >> 1) & 7))];
        if (!live) af[i] = cplx<double>{0.0, 0.0};
      }
#pragma unroll
      for (int j = 0; j < 2; ++j) bf[j] = bs[kk * 64 + wn + j * 16 + fr];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          p1[i][j] = BMfma<double>::mac(af[i].re, bf[j].re, p1[i][j]);
          p1[i][j] = BMfma<double>::mac(-af[i].im, bf[j].im, p1[i][j]);
          p3[i][j] = BMfma<double>::mac(af[i].re, bf[j].im, p3[i][j]);
          p3[i][j] = BMfma<double>::mac(af[i].im, bf[j].re, p3[i][j]);
        }
    }
  }
  // the LDS buffers are free again once every wavefront has read the last stage
  __syncthreads();
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    cplx<double> cv[4][2];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int gr = min(m0 + wm + i * 16 + BMfma<double>::d_row(lane, r), M - 1);
#pragma unroll
      for (int j = 0; j < 2; ++j) cv[r][j] = C[(long)gr * ldc + min(n0 + wn + j * 16 + fr, N - 1)];
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int gr = m0 + wm + i * 16 + BMfma<double>::d_row(lane, r);
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int gc = n0 + wn + j * 16 + fr;
        cplx<double> c = cv[r][j];
        c.re -= p1[i][j][r];
        c.im -= p3[i][j][r];
        if (gr < M && gc < N) C[(long)gr * ldc + gc] = c;
      }
    }
  }
}
constexpr size_t kDirect64TileLds = (size_t)2 * 2 * 64 * 8 * sizeof(cplx<double>);  // 32 KB

// FP32 form for operands whose rows are 16-byte aligned (even leading
// dimension and block offsets, K and N even): 16-byte chunks of two complex
// staged by direct global->LDS loads in stages of 16, two buffers (32 KB).
// A is row-major [64][16] with the chunk at position p of row r stored at
// p ^ (r/2 mod 8), B row-major [16][64]; 3M products as in tile_gemm_sub.
// Chunks past K or N read clamped in-bounds chunks; A values past K are
// zeroed before their products.
__device__ __forceinline__ void tile_gemm_sub_direct32(int m0, int n0, int M, int N, int K,
                                                       const cplx<float> *__restrict__ A, long lda,
                                                       const cplx<float> *__restrict__ B, long ldb,
                                                       cplx<float> *__restrict__ C, long ldc, cplx<float> *smem) {
  typedef BMfma<float>::v4 v4;
  constexpr int BK = 16, NBUF = 2, ASZ = 64 * BK, BSZ = BK * 64;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  const int fr = lane & 15, fk = lane >> 4;
  const cplx<float> *arow[2], *bcol[2];
  int ak[2], bk[2];
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const int c = (wave * 2 + i) * 64 + lane;
    const int row = c >> 3, pos = c & 7;
    arow[i] = A + (long)min(m0 + row, M - 1) * lda;
    ak[i] = 2 * (pos ^ ((row >> 1) & 7));
    const int kr = c >> 5, cp = c & 31;
    bcol[i] = B + min(n0 + 2 * cp, N - 2);
    bk[i] = kr;
  }
  const unsigned lds0 = (unsigned)(size_t)(const __attribute__((address_space(3))) void *)smem;
  auto issue = [&](int buf, int k0) {
#pragma unroll
    for (int i = 0; i < 2; ++i)
      lds_direct_load16(lds0 + (unsigned)((buf * ASZ + (wave * 2 + i) * 128) * sizeof(cplx<float>)),
                        arow[i] + min(k0 + ak[i], K - 2));
#pragma unroll
    for (int i = 0; i < 2; ++i)
      lds_direct_load16(lds0 + (unsigned)((NBUF * ASZ + buf * BSZ + (wave * 2 + i) * 128) * sizeof(cplx<float>)),
                        bcol[i] + (long)min(k0 + bk[i], K - 1) * ldb);
  };
  v4 p1[2][2], p2[2][2], p3[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) p1[i][j] = p2[i][j] = p3[i][j] = v4{0, 0, 0, 0};
  const int nk = (K + BK - 1) / BK;
  if (nk > 0) issue(0, 0);
  for (int kt = 0; kt < nk; ++kt) {
    wait_vmcnt<0>();
    __syncthreads();
    if (kt + 1 < nk) issue((kt + 1) & 1, (kt + 1) * BK);
    const cplx<float> *as = smem + (kt & 1) * ASZ;
    const cplx<float> *bs = smem + NBUF * ASZ + (kt & 1) * BSZ;
#pragma unroll
    for (int ks = 0; ks < BK; ks += 4) {
      const int kk = ks + fk;
      const bool live = kt * BK + kk < K;
      cplx<float> af[2], bf[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        const int row = wm + i * 16 + fr;
        af[i] = as[row * BK + 2 * ((kk >> 1) ^ ((row >> 1) & 7)) + (kk & 1)];
        if (!live) af[i] = cplx<float>{0.f, 0.f};
      }
#pragma unroll
      for (int j = 0; j < 2; ++j) bf[j] = bs[kk * 64 + wn + j * 16 + fr];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          p1[i][j] = BMfma<float>::mac(af[i].re, bf[j].re, p1[i][j]);
          p2[i][j] = BMfma<float>::mac(af[i].im, bf[j].im, p2[i][j]);
          p3[i][j] = BMfma<float>::mac(af[i].re + af[i].im, bf[j].re + bf[j].im, p3[i][j]);
        }
    }
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    cplx<float> cv[4][2];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int gr = min(m0 + wm + i * 16 + BMfma<float>::d_row(lane, r), M - 1);
#pragma unroll
      for (int j = 0; j < 2; ++j) cv[r][j] = C[(long)gr * ldc + min(n0 + wn + j * 16 + fr, N - 1)];
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int gr = m0 + wm + i * 16 + BMfma<float>::d_row(lane, r);
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int gc = n0 + wn + j * 16 + fr;
        cplx<float> c = cv[r][j];
        c.re -= p1[i][j][r] - p2[i][j][r];
        c.im -= p3[i][j][r] - p1[i][j][r] - p2[i][j][r];
        if (gr < M && gc < N) C[(long)gr * ldc + gc] = c;
      }
    }
  }
}

// All of C[M x N] -= A[M x K] B[K x N] by one workgroup, tile after tile.
template <typename T>
__device__ void wg_gemm_sub(int M, int N, int K, const cplx<T> *__restrict__ A, long lda,
                            const cplx<T> *__restrict__ B, long ldb, cplx<T> *__restrict__ C, long ldc,
                            cplx<T> *As, cplx<T> *Bs) {
  const int tm = (M + 63) / 64, tn = (N + 63) / 64;
  for (int t = 0; t < tm * tn; ++t) tile_gemm_sub<T>((t / tn) * 64, (t % tn) * 64, M, N, K, A, lda, B, ldb, C, ldc, As, Bs);
}

// Workgroup argmax of (v, row): largest v, smallest row on ties; every
// thread returns the result.
template <typename T>
__device__ __forceinline__ void wg_argmax(T &v, int &r, T *sv, int *sr) {
  for (int off = 32; off > 0; off >>= 1) {
    const T ov = __shfl_xor(v, off);
    const int orow = __shfl_xor(r, off);
    if (ov > v || (ov == v && orow < r)) {
      v = ov;
      r = orow;
    }
  }
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  __syncthreads();
  if (lane == 0) {
    sv[wave] = v;
    sr[wave] = r;
  }
  __syncthreads();
  v = sv[0];
  r = sr[0];
  for (int w = 1; w < 4; ++w)
    if (sv[w] > v || (sv[w] == v && sr[w] < r)) {
      v = sv[w];
      r = sr[w];
    }
  __syncthreads();
}

__device__ __forceinline__ int item_n(const hp_batch_item &it) { return it.sys.nc * it.sys.nr; }

// Next system of a persistent grid (all threads get the same index).
__device__ __forceinline__ int next_item(unsigned *counter, int *s_idx) {
  if (threadIdx.x == 0) *s_idx = (int)atomicAdd(counter, 1u);
  __syncthreads();
  const int idx = *s_idx;
  __syncthreads();
  return idx;
}

__global__ void batch_zero_kernel(unsigned *p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0u;
}

// ---------------------------------------------------------------- assembly --
// Assembly of every system's C(E) (as hp_build_matrix, Eq. block_structure,
// with a non-local system's sqrt(w_i w_j) W_cc'(r_i, r_j) on every element):
// rows spread over kBuildGroups workgroups per system so that a bucket's
// matrices are written by thousands of workgroups at once.
constexpr int kBuildGroups = 64;
template <typename T>
__global__ __launch_bounds__(256) void batch_build_kernel(int count, const hp_batch_item *__restrict__ items,
                                                          cplx<T> *__restrict__ A) {
  // kBuildGroups workgroups per system (blockIdx.y), each taking every
  // kBuildGroups-th row
  const int s = blockIdx.y;
  if (s >= count) return;
  const hp_batch_item it = items[s];
  const int nc = it.sys.nc, nr = it.sys.nr, n = nc * nr;
  const double h = it.sys.hbar2_2mu, E = it.E;
  const cplx<double> *W = reinterpret_cast<const cplx<double> *>(it.sys.vnl);  // null: local
  cplx<T> *a = A + it.a_off;
  for (int row = blockIdx.x; row < n; row += gridDim.x) {
    const int c = row / nr, i = row - c * nr;
    const int lc = it.sys.l[c];
    const double ri = it.sys.r[i];
    const double diag = h * (double)lc * (double)(lc + 1) / (ri * ri) + it.sys.eps[c] - E;
    const double *tl_row = it.sys.tl + (size_t)i * nr;
    const double *v_row = it.sys.v + 2 * ((size_t)i * nc + c) * nc;
    const double si = W ? sqrt(it.sys.w[i]) : 0.0;
    for (int col = threadIdx.x; col < n; col += 256) {
      const int cp = col / nr, j = col - cp * nr;
      double re = 0.0, im = 0.0;
      if (cp == c) {
        re = h * tl_row[j];
        if (j == i) re += diag;
      }
      if (j == i) {
        re += v_row[2 * cp];
        im += v_row[2 * cp + 1];
      }
      if (W) {
        const double f = si * sqrt(it.sys.w[j]);
        const cplx<double> x = W[(long)row * n + col];
        re += f * x.re;
        im += f * x.im;
      }
      a[(long)row * n + col] = cplx<T>{(T)re, (T)im};
    }
  }
}

// ----------------------------------------------------------- factorization --
// P A = L U with partial pivoting (largest |Re|+|Im|, smallest row on ties),
// in panels of W columns:
//   column steps: pivot search, full-row interchange, scaling of the column
//   and update of the panel's remaining columns;
//   block row: U12 = L11^-1 A12 (one thread per column);
//   trailing update A22 -= L21 U12 (MFMA tiles).

// Substitution on one diagonal block [b0, b0 + bs) of an LU factor for the
// right-hand column c of y (leading dimension nc): unit lower (forward) or
// upper (backward, dividing by the diagonal).  D: the block in LDS at
// stride LP (kBK + 1 by default), zero past bs.  Rows are taken 8 at a time
// in registers; the rows solved before such a group (above it forward, below
// it backward) are read back from y.  Both solve forms of the batch and the
// block rows of both factorization forms use this routine.
template <typename T, int LP = kBK + 1>
__device__ __forceinline__ void diag_block_solve(const cplx<T> *D, cplx<T> *__restrict__ y, int nc, int b0, int bs,
                                                 int c, bool upper) {
  constexpr int RB = 8;
  const cplx<T> zero{T(0), T(0)};
  const int nb = (bs + RB - 1) / RB;
#pragma unroll 1
  for (int q = 0; q < nb; ++q) {
    const int r0 = (upper ? nb - 1 - q : q) * RB;
    cplx<T> acc[RB];
#pragma unroll
    for (int u = 0; u < RB; ++u) acc[u] = r0 + u < bs ? y[(long)(b0 + r0 + u) * nc + c] : zero;
    const int k0 = upper ? r0 + RB : 0, k1 = upper ? bs : r0;
#pragma unroll 4
    for (int kk = k0; kk < k1; ++kk) {
      const cplx<T> xk = y[(long)(b0 + kk) * nc + c];
#pragma unroll
      for (int u = 0; u < RB; ++u) acc[u] = cfms(acc[u], D[(r0 + u) * LP + kk], xk);
    }
    if (!upper) {
#pragma unroll
      for (int u = 1; u < RB; ++u)
#pragma unroll
        for (int v = 0; v < u; ++v) acc[u] = cfms(acc[u], D[(r0 + u) * LP + r0 + v], acc[v]);
    } else {
#pragma unroll
      for (int u = RB - 1; u >= 0; --u)
        if (r0 + u < bs) {
#pragma unroll
          for (int v = u + 1; v < RB; ++v)
            if (r0 + v < bs) acc[u] = cfms(acc[u], D[(r0 + u) * LP + r0 + v], acc[v]);
          acc[u] = cdiv(acc[u], D[(r0 + u) * LP + r0 + u]);
        }
    }
#pragma unroll
    for (int u = 0; u < RB; ++u)
      if (r0 + u < bs) y[(long)(b0 + r0 + u) * nc + c] = acc[u];
  }
}

// The diagonal block [b0, b0 + bs) of lu (leading dimension n) into D
// (stride kBK + 1, zero-padded to kBK x kBK); the caller synchronizes.
template <typename T>
__device__ __forceinline__ void stage_diag_block(cplx<T> *D, const cplx<T> *__restrict__ lu, int n, int b0, int bs) {
  constexpr int B = kBK, LP = kBK + 1;
  for (int e = threadIdx.x; e < B * B; e += blockDim.x) {
    const int r = e / B, k = e - r * B;
    D[r * LP + k] = (r < bs && k < bs) ? lu[(long)(b0 + r) * n + b0 + k] : cplx<T>{T(0), T(0)};
  }
}

// Column steps of the panel [j0, j0 + w) of one n x n system, by one
// workgroup.  Records the pivots, and the first exactly zero pivot column
// (1-based) in *first_zero if it is still 0.  The candidate of column j + 1
// is found while column j's update writes it (one pass over the panel rows
// per column).  full_rows: every interchange is applied to the whole row at
// once and the block row U12 = L11^-1 A12 over [j0 + w, n) follows (the
// persistent form); otherwise the interchanges touch the panel's columns
// only, and batch_swap_brow_kernel applies them to the other columns and
// forms the block row afterwards (the stepped form).
template <typename T>
__device__ void panel_steps(cplx<T> *a, int n, int j0, int w, bool full_rows, int *piv, int *first_zero,
                            cplx<T> *urow, T *sv, int *sr, cplx<T> *D) {
  const int tid = threadIdx.x;
  T best = T(-1);
  int brow = INT_MAX;
  for (int r = j0 + tid; r < n; r += 256) {
    const T v = cabs1(a[(long)r * n + j0]);
    if (v > best || (v == best && r < brow)) {
      best = v;
      brow = r;
    }
  }
  for (int jj = 0; jj < w; ++jj) {
    const int j = j0 + jj;
    wg_argmax(best, brow, sv, sr);
    const int p = (brow >= j && brow < n) ? brow : j;
    const bool nz = best > T(0);
    if (tid == 0) {
      piv[j] = p;
      if (!nz && *first_zero == 0) *first_zero = j + 1;
    }
    if (p != j) {
      const int c0 = full_rows ? 0 : j0, c1 = full_rows ? n : j0 + w;
      for (int c = c0 + tid; c < c1; c += 256) {
        const cplx<T> x = a[(long)j * n + c];
        a[(long)j * n + c] = a[(long)p * n + c];
        a[(long)p * n + c] = x;
      }
    }
    __syncthreads();
    if (tid < w) urow[tid] = a[(long)j * n + j0 + tid];
    __syncthreads();
    best = T(-1);
    brow = INT_MAX;
    const bool next = jj + 1 < w;
    const cplx<T> inv = nz ? crcp(urow[jj]) : cplx<T>{T(0), T(0)};
    for (int r = j + 1 + tid; r < n; r += 256) {
      cplx<T> *row = a + (long)r * n + j0;
      if (nz) {
        const cplx<T> l = cmul(row[jj], inv);
        row[jj] = l;
        for (int c = jj + 1; c < w; ++c) row[c] = cfms(row[c], l, urow[c]);
      }
      if (next) {
        const T v = cabs1(row[jj + 1]);
        if (v > best || (v == best && r < brow)) {
          best = v;
          brow = r;
        }
      }
    }
    __syncthreads();
  }
  if (!full_rows) return;
  // U12 = L11^-1 A12: L11 staged in LDS (D: kBK x (kBK + 1)), each column
  // of A12 by diag_block_solve (the terms in the same order as a plain
  // substitution)
  stage_diag_block<T>(D, a, n, j0, w);
  __syncthreads();
  for (int c = j0 + w + tid; c < n; c += 256) diag_block_solve<T>(D, a + (long)j0 * n, n, 0, w, c, false);
  __syncthreads();
}

// perm = the composition of the interchanges (one thread).
__device__ void compose_perm(const int *piv, int *pm, int n) {
  for (int i = 0; i < n; ++i) pm[i] = i;
  for (int k = 0; k < n; ++k) {
    const int p = piv[k];
    const int x = pm[k];
    pm[k] = pm[p];
    pm[p] = x;
  }
}

// Persistent form: one workgroup factors one system at a time.
template <typename T>
__global__ __launch_bounds__(256) void batch_lu_kernel(int count, const hp_batch_item *__restrict__ items,
                                                       cplx<T> *__restrict__ A, int *__restrict__ ipiv,
                                                       int *__restrict__ perm, int *__restrict__ info,
                                                       unsigned *counter, int W) {
  extern __shared__ __align__(16) char smem_raw[];
  cplx<T> *As = reinterpret_cast<cplx<T> *>(smem_raw);
  cplx<T> *Bs = As + kBK * kBLd;
  __shared__ cplx<T> urow[kBK];
  __shared__ T sv[4];
  __shared__ int sr[4];
  __shared__ int s_idx;
  __shared__ int s_zero;
  const int tid = threadIdx.x;
  for (;;) {
    const int s = next_item(counter, &s_idx);
    if (s >= count) break;
    const hp_batch_item it = items[s];
    const int n = item_n(it);
    cplx<T> *a = A + it.a_off;
    int *piv = ipiv + it.p_off;
    if (tid == 0) s_zero = 0;
    __syncthreads();
    for (int j0 = 0; j0 < n; j0 += W) {
      const int w = min(W, n - j0);
      panel_steps<T>(a, n, j0, w, true, piv, &s_zero, urow, sv, sr, As);  // As is free until the product
      const int rest = n - j0 - w;
      if (rest > 0)
        wg_gemm_sub<T>(rest, rest, w, a + (long)(j0 + w) * n + j0, n, a + (long)j0 * n + j0 + w, n,
                       a + (long)(j0 + w) * n + j0 + w, n, As, Bs);
    }
    if (tid == 0) {
      compose_perm(piv, perm + it.p_off, n);
      info[s] = s_zero;
    }
    __syncthreads();
  }
}

// Stepped form, for buckets of larger systems, blocked in two levels: outer
// blocks of NB columns (a multiple of the panel width W, at most kBlockMax),
// each factored as NB / W panels whose updates stay inside the block, then
// the block's row U12 = L11^-1 A12 over all columns right of it and one
// trailing update A22 -= L21 U12 with K = NB.  Every step is one launch over
// the systems still factoring (listed largest first, so they are items
// [0, active)): the panels' column steps one workgroup per system, the
// updates and the block row as tiles of all systems.  With NB = W this is
// the one-level blocked LU.
constexpr int kBlockMax = 64;

template <typename T>
__global__ __launch_bounds__(256) void batch_panel_kernel(const hp_batch_item *__restrict__ items,
                                                          cplx<T> *__restrict__ A, int *__restrict__ ipiv,
                                                          int *__restrict__ perm, int *__restrict__ info, int j0,
                                                          int W, int NB) {
  __shared__ cplx<T> urow[kBK];
  __shared__ cplx<T> D[kBK * (kBK + 1)];
  __shared__ T sv[4];
  __shared__ int sr[4];
  __shared__ int s_zero;
  const int s = blockIdx.x;
  const hp_batch_item it = items[s];
  const int n = item_n(it);
  if (j0 >= n) return;
  const int w = min(W, n - j0);
  (void)NB;
  int *piv = ipiv + it.p_off;
  if (threadIdx.x == 0) s_zero = info[s];
  __syncthreads();
  panel_steps<T>(A + it.a_off, n, j0, w, false, piv, &s_zero, urow, sv, sr, D);
  if (threadIdx.x == 0) {
    info[s] = s_zero;
    if (j0 + w == n) compose_perm(piv, perm + it.p_off, n);
  }
}

// The same column steps with the panel held in registers: one workgroup of
// 1024 threads per system, thread t owning panel rows j0 + t + 1024 k
// (k < RPT, so n - j0 <= 1024 RPT) with their W columns.  Per column: the
// pivot search over the registers, a workgroup argmax, the interchange of the
// two rows through LDS, the pivot row broadcast in LDS, and the update of the
// rows below in registers; the panel is read and written once instead of
// once per column.  Same arithmetic as panel_steps (interchanges inside the
// panel only).
constexpr int kRegPanelThreads = 1024;
std::atomic<int> g_reg_panel{1};  // hp_set_batch_reg_panel
template <typename T, int W, int RPT>
__global__ __launch_bounds__(kRegPanelThreads) void batch_panel_reg_kernel(
    const hp_batch_item *__restrict__ items, cplx<T> *__restrict__ A, int *__restrict__ ipiv,
    int *__restrict__ perm, int *__restrict__ info, int j0) {
  constexpr int NW = kRegPanelThreads / 64;
  __shared__ cplx<T> prow[W], jrow[W];
  __shared__ T sv[NW];
  __shared__ int sr[NW];
  __shared__ int s_zero;
  const int s = blockIdx.x;
  const hp_batch_item it = items[s];
  const int n = item_n(it);
  if (j0 >= n) return;
  const int w = min(W, n - j0);
  cplx<T> *a = A + it.a_off;
  int *piv = ipiv + it.p_off;
  const int tid = threadIdx.x;
  if (tid == 0) s_zero = info[s];
  cplx<T> P[RPT][W];
#pragma unroll
  for (int k = 0; k < RPT; ++k) {
    const int r = j0 + tid + k * kRegPanelThreads;
#pragma unroll
    for (int c = 0; c < W; ++c)
      P[k][c] = (r < n && c < w) ? a[(long)r * n + j0 + c] : cplx<T>{T(0), T(0)};
  }
  __syncthreads();
#pragma unroll
  for (int jj = 0; jj < W; ++jj) {
    if (jj >= w) break;  // uniform
    const int j = j0 + jj;
    T best = T(-1);
    int brow = INT_MAX;
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
      const int r = j0 + tid + k * kRegPanelThreads;
      if (r >= j && r < n) {
        const T v = cabs1(P[k][jj]);
        if (v > best || (v == best && r < brow)) {
          best = v;
          brow = r;
        }
      }
    }
    for (int off = 32; off > 0; off >>= 1) {
      const T ov = __shfl_xor(best, off);
      const int orow = __shfl_xor(brow, off);
      if (ov > best || (ov == best && orow < brow)) {
        best = ov;
        brow = orow;
      }
    }
    if ((tid & 63) == 0) {
      sv[tid >> 6] = best;
      sr[tid >> 6] = brow;
    }
    __syncthreads();
    best = sv[0];
    brow = sr[0];
#pragma unroll
    for (int q = 1; q < NW; ++q)
      if (sv[q] > best || (sv[q] == best && sr[q] < brow)) {
        best = sv[q];
        brow = sr[q];
      }
    const int p = (brow >= j && brow < n) ? brow : j;
    const bool nz = best > T(0);
    if (tid == 0) {
      piv[j] = p;
      if (!nz && s_zero == 0) s_zero = j + 1;
    }
    // rows j and p: the pivot row to prow (the new row j), row j to jrow
    const int oj = j - j0, op = p - j0;
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
      const int r = tid + k * kRegPanelThreads;
      if (r == op) {
#pragma unroll
        for (int c = 0; c < W; ++c) prow[c] = P[k][c];
      }
      if (r == oj && op != oj) {
#pragma unroll
        for (int c = 0; c < W; ++c) jrow[c] = P[k][c];
      }
    }
    __syncthreads();
    if (op != oj) {
#pragma unroll
      for (int k = 0; k < RPT; ++k) {
        const int r = tid + k * kRegPanelThreads;
        if (r == oj) {
#pragma unroll
          for (int c = 0; c < W; ++c) P[k][c] = prow[c];
        }
        if (r == op) {
#pragma unroll
          for (int c = 0; c < W; ++c) P[k][c] = jrow[c];
        }
      }
    }
    if (nz) {
      const cplx<T> inv = crcp(prow[jj]);
#pragma unroll
      for (int k = 0; k < RPT; ++k) {
        const int r = j0 + tid + k * kRegPanelThreads;
        if (r > j && r < n) {
          const cplx<T> l = cmul(P[k][jj], inv);
          P[k][jj] = l;
#pragma unroll
          for (int c = jj + 1; c < W; ++c) P[k][c] = cfms(P[k][c], l, prow[c]);
        }
      }
    }
    __syncthreads();  // prow and jrow are rewritten by the next column
  }
#pragma unroll
  for (int k = 0; k < RPT; ++k) {
    const int r = j0 + tid + k * kRegPanelThreads;
    if (r < n) {
#pragma unroll
      for (int c = 0; c < W; ++c)
        if (c < w) a[(long)r * n + j0 + c] = P[k][c];
    }
  }
  if (tid == 0) {
    info[s] = s_zero;
    if (j0 + w == n) compose_perm(piv, perm + it.p_off, n);
  }
}

// Shapes of the tiled steps of one system (n) at one step:
//   kind 0, inner update after the panel at j0: rows [j0 + w, n) x columns
//     [j0 + w, end of the outer block), K = w;
//   kind 1, outer update of the block at J: rows and columns [J + NB, n), K = NB;
//   kind 2, block row of the block at J: columns [J + NB, n) in chunks of 256;
//   kind 3, after the panel at j0: its interchanges on every column outside
//     the panel, and the panel's block row over [j0 + w, end of the outer
//     block), columns in chunks of 256.
struct StepShape {
  int r0, rows, c0, cols, k0, K;
};
__device__ __host__ inline StepShape step_shape(int kind, int n, int j, int W, int NB) {
  StepShape sh{0, 0, 0, 0, 0, 0};
  if (j >= n) return sh;
  if (kind == 0) {
    const int w = min(W, n - j);
    const int cend = min((j / NB + 1) * NB, n);
    sh.r0 = sh.c0 = j + w;
    sh.rows = n - sh.r0;
    sh.cols = cend - sh.c0;
    sh.k0 = j;
    sh.K = w;
  } else {
    const int nb = min(NB, n - j);
    sh.r0 = sh.c0 = j + nb;
    sh.rows = sh.cols = n - sh.r0;
    sh.k0 = j;
    sh.K = nb;
  }
  return sh;
}
__device__ __host__ inline int step_units(int kind, int n, int j, int W, int NB) {
  if (kind == 3) return j < n ? (n - min(W, n - j) + 255) / 256 : 0;
  const StepShape sh = step_shape(kind, n, j, W, NB);
  if (sh.rows <= 0 || sh.cols <= 0) return 0;
  if (kind == 2) return (sh.cols + 255) / 256;
  return ((sh.rows + 63) / 64) * ((sh.cols + 63) / 64);
}

// Work-unit offsets of every tiled step: offs[q * (count + 1) + s] = units of
// systems [0, s) at step q (exclusive prefix sum).  Steps q < P are the inner
// updates after the panels at j = q W, steps P <= q < 2P their interchange
// and block-row steps; then, per outer block b (J = b NB), the block row
// (2P + 2b) and the outer update (2P + 2b + 1).
__global__ void batch_tables_kernel(int count, const hp_batch_item *__restrict__ items, int W, int NB, int P,
                                    int *offs) {
  const int q = blockIdx.x;
  if (threadIdx.x != 0) return;
  int kind, j;
  if (q < P) {
    kind = 0;
    j = q * W;
  } else if (q < 2 * P) {
    kind = 3;
    j = (q - P) * W;
  } else {
    kind = ((q - 2 * P) & 1) ? 1 : 2;
    j = ((q - 2 * P) >> 1) * NB;
  }
  int acc = 0;
  int *o = offs + (long)q * (count + 1);
  for (int s = 0; s < count; ++s) {
    o[s] = acc;
    acc += step_units(kind, item_n(items[s]), j, W, NB);
  }
  o[count] = acc;
}

// The system owning unit g of a step: offs[s] <= g < offs[s + 1].
__device__ __forceinline__ int unit_owner(const int *offs, int count, int g) {
  int lo = 0, hi = count;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (offs[mid] <= g)
      lo = mid;
    else
      hi = mid;
  }
  return lo;
}

// The update tiles of one step (kind 0 or 1) of every system.
template <typename T>
__global__ __launch_bounds__(256) void batch_trail_kernel(int count, const hp_batch_item *__restrict__ items,
                                                          cplx<T> *__restrict__ A, const int *__restrict__ offs,
                                                          int kind, int j, int W, int NB) {
  extern __shared__ __align__(16) char smem_raw[];
  cplx<T> *As = reinterpret_cast<cplx<T> *>(smem_raw);
  cplx<T> *Bs = As + kBK * kBLd;
  const int g = blockIdx.x;
  if (g >= offs[count]) return;
  const int s = unit_owner(offs, count, g);
  const hp_batch_item it = items[s];
  const int n = item_n(it);
  const StepShape sh = step_shape(kind, n, j, W, NB);
  const int tn = (sh.cols + 63) / 64;
  const int l = g - offs[s];
  cplx<T> *a = A + it.a_off;
  const cplx<T> *pa = a + (long)sh.r0 * n + sh.k0, *pb = a + (long)sh.k0 * n + sh.c0;
  cplx<T> *pc = a + (long)sh.r0 * n + sh.c0;
  if constexpr (std::is_same<T, double>::value) {
    tile_gemm_sub_direct64((l / tn) * 64, (l % tn) * 64, sh.rows, sh.cols, sh.K, pa, n, pb, n, pc, n, As);
  } else {
    // direct staging needs 16-byte aligned rows and chunks that never
    // straddle the end of K or of a row (uniform over the workgroup)
    const bool aligned = (n % 2 == 0) && (sh.K % 2 == 0) && (sh.cols % 2 == 0) &&
                         ((((uintptr_t)pa) | ((uintptr_t)pb)) & 15) == 0;
    if (aligned)
      tile_gemm_sub_direct32((l / tn) * 64, (l % tn) * 64, sh.rows, sh.cols, sh.K, pa, n, pb, n, pc, n, As);
    else
      tile_gemm_sub<T>((l / tn) * 64, (l % tn) * 64, sh.rows, sh.cols, sh.K, pa, n, pb, n, pc, n, As, Bs);
  }
}

// After the panel at j of every system (kind 3 units): the panel's
// interchanges on every column outside it, 256 columns per workgroup, one per
// thread, in the order they were chosen; for the columns [j + w, end of the
// outer block) then the panel's block row by diag_block_solve with the
// panel's L11 staged in LDS.
template <typename T>
__global__ __launch_bounds__(256) void batch_swap_brow_kernel(int count, const hp_batch_item *__restrict__ items,
                                                              cplx<T> *__restrict__ A, const int *__restrict__ ipiv,
                                                              const int *__restrict__ offs, int j, int W, int NB) {
  __shared__ cplx<T> D[kBK * (kBK + 1)];
  __shared__ int sp[kBK];
  const int g = blockIdx.x;
  if (g >= offs[count]) return;
  const int s = unit_owner(offs, count, g);
  const hp_batch_item it = items[s];
  const int n = item_n(it);
  const int w = min(W, n - j);
  const int cend = min((j / NB + 1) * NB, n);
  cplx<T> *a = A + it.a_off;
  const int *piv = ipiv + it.p_off;
  if (threadIdx.x < w) sp[threadIdx.x] = piv[j + threadIdx.x];
  stage_diag_block<T>(D, a, n, j, w);
  __syncthreads();
  const int x = (g - offs[s]) * 256 + (int)threadIdx.x;
  if (x >= n - w) return;
  const int c = x < j ? x : x + w;
  for (int k = 0; k < w; ++k) {
    const int p = sp[k];
    if (p != j + k) {
      const cplx<T> v = a[(long)(j + k) * n + c];
      a[(long)(j + k) * n + c] = a[(long)p * n + c];
      a[(long)p * n + c] = v;
    }
  }
  if (c >= j + w && c < cend) diag_block_solve<T>(D, a + (long)j * n, n, 0, w, c, false);
}

// Block row of the outer block at J of every system: U12 = L11^-1 A12 over
// the columns [J + nb, n), 256 columns per workgroup, one per thread; L11
// (unit lower, nb x nb) staged in LDS (zero past nb), the substitution by
// diag_block_solve.
template <typename T>
__global__ __launch_bounds__(256) void batch_brow_kernel(int count, const hp_batch_item *__restrict__ items,
                                                         cplx<T> *__restrict__ A, const int *__restrict__ offs,
                                                         int J, int NB) {
  // every lane reads the same element of D (a broadcast), so no padding
  constexpr int LP = kBlockMax;
  __shared__ cplx<T> D[kBlockMax * LP];
  const int g = blockIdx.x;
  if (g >= offs[count]) return;
  const int s = unit_owner(offs, count, g);
  const hp_batch_item it = items[s];
  const int n = item_n(it);
  const int nb = min(NB, n - J);
  cplx<T> *a = A + it.a_off;
  const int nbp = (nb + 7) & ~7;  // rows of the last 8-row group
  for (int e = threadIdx.x; e < nbp * nb; e += 256) {
    const int r = e / nb, k = e - r * nb;
    D[r * LP + k] = r < nb ? a[(long)(J + r) * n + J + k] : cplx<T>{T(0), T(0)};
  }
  __syncthreads();
  const int c = J + nb + (g - offs[s]) * 256 + (int)threadIdx.x;
  if (c >= n) return;
  diag_block_solve<T, LP>(D, a + (long)J * n, n, 0, nb, c, false);
}

// ------------------------------------------------------------------- solves --
// Y (n x nc, leading dimension nc) <- U^-1 L^-1 Y in place, blocks of kBK rows:
// the diagonal block by substitution (one thread per column), the rows
// beyond it by a workgroup GEMM.
template <typename T>
__device__ void wg_lu_solve(int n, int nc, const cplx<T> *__restrict__ lu, cplx<T> *__restrict__ y, cplx<T> *As,
                            cplx<T> *Bs) {
  const int tid = threadIdx.x;
  static_assert(kBK * kBLd >= kBK * (kBK + 1), "the diagonal block fits the A tile");
  for (int b = 0; b < n; b += kBK) {
    const int bs = min(kBK, n - b);
    __syncthreads();  // As is free (the previous step's product is done with it)
    stage_diag_block<T>(As, lu, n, b, bs);
    __syncthreads();
    for (int c = tid; c < nc; c += 256) diag_block_solve<T>(As, y, nc, b, bs, c, false);
    __syncthreads();
    if (b + bs < n)
      wg_gemm_sub<T>(n - b - bs, nc, bs, lu + (long)(b + bs) * n + b, n, y + (long)b * nc, nc,
                     y + (long)(b + bs) * nc, nc, As, Bs);
  }
  const int nb = (n + kBK - 1) / kBK;
  for (int bi = nb - 1; bi >= 0; --bi) {
    const int b = bi * kBK, bs = min(kBK, n - b);
    __syncthreads();
    stage_diag_block<T>(As, lu, n, b, bs);
    __syncthreads();
    for (int c = tid; c < nc; c += 256) diag_block_solve<T>(As, y, nc, b, bs, c, true);
    __syncthreads();
    if (b > 0)
      wg_gemm_sub<T>(b, nc, bs, lu + b, n, y + (long)b * nc, nc, y, nc, As, Bs);
  }
}

// Per-system refinement state.
struct BatchState {
  int status;  // 0 running, 1 converged, 2 not converged, 3 zero pivot, 4 unsupported
  int iters;
  double corr_prev;
  double corr;
};

// mode 0: Y = P B (B[(c,i)][c'] = delta_cc' q_i) and solve; then X = Y (FP64)
// mode 1: Y = P R / s (per column, R the FP64 residual, s its column max) and
//         solve, for systems still refining.
template <typename T>
__global__ __launch_bounds__(256) void batch_solve_kernel(int count, const hp_batch_item *__restrict__ items,
                                                          const cplx<T> *__restrict__ LU,
                                                          const int *__restrict__ perm, cplx<T> *__restrict__ Y,
                                                          cplx<double> *__restrict__ X,
                                                          const cplx<double> *__restrict__ Rr,
                                                          const double *__restrict__ cscale,
                                                          BatchState *state, int mode) {
  extern __shared__ __align__(16) char smem_raw[];
  cplx<T> *As = reinterpret_cast<cplx<T> *>(smem_raw);
  cplx<T> *Bs = As + kBK * kBLd;
  const int s = blockIdx.x;
  if (s >= count) return;
  const hp_batch_item it = items[s];
  if (mode == 1 && state[s].status != 0) return;
  const int nc = it.sys.nc, nr = it.sys.nr, n = nc * nr;
  const int *pm = perm + it.p_off;
  cplx<T> *y = Y + it.x_off;
  const long cnt = (long)n * nc;
  for (long e = threadIdx.x; e < cnt; e += 256) {
    const int i = (int)(e / nc), cc = (int)(e - (long)i * nc);
    const int src = pm[i];
    cplx<T> v{T(0), T(0)};
    if (mode == 0) {
      const int c = src / nr, ii = src - c * nr;
      if (c == cc) v.re = (T)it.sys.q[ii];
    } else {
      const cplx<double> r = Rr[it.x_off + (long)src * nc + cc];
      const double sc = cscale[it.c_off + cc];
      v = cplx<T>{(T)(r.re / sc), (T)(r.im / sc)};
    }
    y[e] = v;
  }
  __syncthreads();
  wg_lu_solve<T>(n, nc, LU + it.a_off, y, As, Bs);
  if (mode == 0 && X)
    for (long e = threadIdx.x; e < cnt; e += 256) X[it.x_off + e] = cplx<double>{(double)y[e].re, (double)y[e].im};
}

// R = B - C X in FP64 from the block structure, and per column s = max |R|
// (|Re|+|Im|; 1 for an exactly zero column), for systems still refining,
// spread over kResChunks workgroups per system (grid kResChunks x count):
// R = h (T + L) X + diagonal term (pass 1, RB1 mesh rows of one channel per
// item), then R = B - (R + V_i X_i) (pass 2, RB2 channels at one mesh point
// per item) with the column maxima gathered by atomics into cscale (as the
// bits of non-negative doubles), then the maxima turned into scales.  Every
// output element keeps the summation order of the definition (kinetic terms
// over j, the diagonal term, coupling terms over c').
constexpr int kResChunks = 64;

__global__ __launch_bounds__(256) void batch_res_kinetic_kernel(int count, const hp_batch_item *__restrict__ items,
                                                                const cplx<double> *__restrict__ X,
                                                                cplx<double> *__restrict__ Rr, double *cscale,
                                                                const BatchState *state) {
  constexpr int RB1 = 8;
  const int s = blockIdx.y;
  if (s >= count || state[s].status != 0) return;
  const hp_batch_item it = items[s];
  const int nc = it.sys.nc, nr = it.sys.nr;
  const double h = it.sys.hbar2_2mu, E = it.E;
  const cplx<double> *x = X + it.x_off;
  cplx<double> *rr = Rr + it.x_off;
  if (blockIdx.x == 0)
    for (int c = threadIdx.x; c < nc; c += 256) cscale[it.c_off + c] = 0.0;  // pass 2 gathers maxima here
  const int nrb = (nr + RB1 - 1) / RB1;
  const long n1 = (long)nc * nrb * nc;
  for (long e = (long)blockIdx.x * 256 + threadIdx.x; e < n1; e += (long)kResChunks * 256) {
    const int cc = (int)(e % nc);
    const long t = e / nc;
    const int ib = (int)(t % nrb), c = (int)(t / nrb);
    const int i0 = ib * RB1;
    const cplx<double> *xc = x + (long)c * nr * nc + cc;
    double sr[RB1], si[RB1];
#pragma unroll
    for (int u = 0; u < RB1; ++u) sr[u] = si[u] = 0.0;
    for (int j = 0; j < nr; ++j) {
      const cplx<double> xv = xc[(long)j * nc];
#pragma unroll
      for (int u = 0; u < RB1; ++u) {
        const int i = min(i0 + u, nr - 1);  // rows past nr: computed, never stored
        const double ht = h * it.sys.tl[(size_t)i * nr + j];
        sr[u] += ht * xv.re;
        si[u] += ht * xv.im;
      }
    }
    const int lc = it.sys.l[c];
#pragma unroll
    for (int u = 0; u < RB1; ++u) {
      const int i = i0 + u;
      if (i < nr) {
        const double ri = it.sys.r[i];
        const double dg = h * (double)lc * (double)(lc + 1) / (ri * ri) + it.sys.eps[c] - E;
        const cplx<double> xi = xc[(long)i * nc];
        rr[((long)c * nr + i) * nc + cc] = cplx<double>{sr[u] + dg * xi.re, si[u] + dg * xi.im};
      }
    }
  }
}

// Non-local systems: rr[(c,i)][cc] += sqrt(w_i) sum over (c',j) of
// W[(c,i),(c',j)] sqrt(w_j) x[(c',j)][cc], between the kinetic pass and the
// coupling pass (which forms b - the sum).  One output per thread, threads
// of a wavefront on consecutive right-hand columns (coalesced x reads, W
// broadcast); sqrt(w) of the mesh in LDS.
constexpr int kNlMaxPoints = 1024;
__global__ __launch_bounds__(256) void batch_res_nonlocal_kernel(int count, const hp_batch_item *__restrict__ items,
                                                                 const cplx<double> *__restrict__ X,
                                                                 cplx<double> *__restrict__ Rr,
                                                                 const BatchState *state) {
  __shared__ double sw[kNlMaxPoints];
  const int s = blockIdx.y;
  if (s >= count || state[s].status != 0) return;
  const hp_batch_item it = items[s];
  if (!it.sys.vnl || it.sys.nr > kNlMaxPoints) return;  // the latter: status 4, never refining
  const int nc = it.sys.nc, nr = it.sys.nr;
  const long n = (long)nc * nr;
  const cplx<double> *W = reinterpret_cast<const cplx<double> *>(it.sys.vnl);
  const cplx<double> *x = X + it.x_off;
  cplx<double> *rr = Rr + it.x_off;
  for (int j = threadIdx.x; j < nr; j += 256) sw[j] = sqrt(it.sys.w[j]);
  __syncthreads();
  for (long e = (long)blockIdx.x * 256 + threadIdx.x; e < n * nc; e += (long)kResChunks * 256) {
    const long row = e / nc;
    const int cc = (int)(e - row * nc);
    const cplx<double> *wr = W + row * n;
    double ar = 0.0, ai = 0.0;
    for (int cp = 0; cp < nc; ++cp) {
      const cplx<double> *wb = wr + (long)cp * nr;
      const cplx<double> *xb = x + (long)cp * nr * nc + cc;
      for (int j = 0; j < nr; ++j) {
        const cplx<double> wv = wb[j];
        const cplx<double> xv = xb[(long)j * nc];
        const double f = sw[j];
        ar += f * (wv.re * xv.re - wv.im * xv.im);
        ai += f * (wv.re * xv.im + wv.im * xv.re);
      }
    }
    const double si = sw[(int)(row % nr)];
    cplx<double> p = rr[e];
    p.re += si * ar;
    p.im += si * ai;
    rr[e] = p;
  }
}

__global__ __launch_bounds__(256) void batch_res_coupling_kernel(int count, const hp_batch_item *__restrict__ items,
                                                                 const cplx<double> *__restrict__ X,
                                                                 cplx<double> *__restrict__ Rr, double *cscale,
                                                                 const BatchState *state) {
  constexpr int RB2 = 4;
  const int s = blockIdx.y;
  if (s >= count || state[s].status != 0) return;
  const hp_batch_item it = items[s];
  const int nc = it.sys.nc, nr = it.sys.nr;
  const cplx<double> *x = X + it.x_off;
  cplx<double> *rr = Rr + it.x_off;
  unsigned long long *cmax = reinterpret_cast<unsigned long long *>(cscale + it.c_off);
  const int ncb = (nc + RB2 - 1) / RB2;
  const long n2 = (long)nr * ncb * nc;
  for (long e = (long)blockIdx.x * 256 + threadIdx.x; e < n2; e += (long)kResChunks * 256) {
    const int cc = (int)(e % nc);
    const long t = e / nc;
    const int cb = (int)(t % ncb), i = (int)(t / ncb);
    const int c0 = cb * RB2;
    const double *vi_ = it.sys.v + 2 * (size_t)i * nc * nc;  // V_i[c][c']
    double sr[RB2], si[RB2];
#pragma unroll
    for (int u = 0; u < RB2; ++u) {
      const int c = min(c0 + u, nc - 1);  // channels past nc: computed, never stored
      const cplx<double> p = rr[((long)c * nr + i) * nc + cc];
      sr[u] = p.re;
      si[u] = p.im;
    }
    for (int cp = 0; cp < nc; ++cp) {
      const cplx<double> xv = x[((long)cp * nr + i) * nc + cc];
#pragma unroll
      for (int u = 0; u < RB2; ++u) {
        const int c = min(c0 + u, nc - 1);
        const double vr = vi_[2 * ((size_t)c * nc + cp)], vim = vi_[2 * ((size_t)c * nc + cp) + 1];
        sr[u] += vr * xv.re - vim * xv.im;
        si[u] += vr * xv.im + vim * xv.re;
      }
    }
    double m = 0.0;
#pragma unroll
    for (int u = 0; u < RB2; ++u) {
      const int c = c0 + u;
      if (c < nc) {
        const double b = (c == cc) ? it.sys.q[i] : 0.0;
        const cplx<double> out{b - sr[u], -si[u]};
        rr[((long)c * nr + i) * nc + cc] = out;
        m = fmax(m, cabs1(out));
      }
    }
    atomicMax(&cmax[cc], (unsigned long long)__double_as_longlong(m));
  }
}

__global__ void batch_res_scale_kernel(int count, const hp_batch_item *__restrict__ items, double *cscale,
                                       const BatchState *state) {
  const int s = blockIdx.x;
  if (s >= count || state[s].status != 0) return;
  const hp_batch_item it = items[s];
  for (int c = threadIdx.x; c < it.sys.nc; c += blockDim.x) {
    const double m = cscale[it.c_off + c];  // the maximum's bits, read as the double they encode
    cscale[it.c_off + c] = (m > 0.0) ? m : 1.0;
  }
}

// X += s Y for systems still refining; relative correction
// corr = max_c |d_c|_inf / |x_c|_inf and the stop rule of hp_solve; counts
// the systems still refining in *active.
template <typename T>
__global__ __launch_bounds__(256) void batch_update_kernel(int count, const hp_batch_item *__restrict__ items,
                                                           const cplx<T> *__restrict__ Y,
                                                           cplx<double> *__restrict__ X,
                                                           const double *__restrict__ cscale, BatchState *state,
                                                           double tol, int max_refine, unsigned *active) {
  __shared__ double red[256];
  const int s = blockIdx.x;
  if (s >= count || state[s].status != 0) return;
  const hp_batch_item it = items[s];
  const int nc = it.sys.nc, n = nc * it.sys.nr;
  const cplx<T> *y = Y + it.x_off;
  cplx<double> *x = X + it.x_off;
  double corr = 0.0;
  for (int cc = threadIdx.x; cc < nc; cc += 256) {
    const double sc = cscale[it.c_off + cc];
    double dm = 0.0, xm = 0.0;
    for (int row = 0; row < n; ++row) {
      const long e = (long)row * nc + cc;
      const cplx<double> d{(double)y[e].re * sc, (double)y[e].im * sc};
      cplx<double> v = x[e];
      v.re += d.re;
      v.im += d.im;
      x[e] = v;
      dm = fmax(dm, cabs1(d));
      xm = fmax(xm, cabs1(v));
    }
    corr = fmax(corr, xm > 0.0 ? dm / xm : dm);
  }
  red[threadIdx.x] = corr;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < off) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + off]);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    BatchState st = state[s];
    corr = red[0];
    st.iters += 1;
    const double corr_tol = tol > 0.0 ? tol : kRefineTol;
    if (corr <= corr_tol) {
      st.status = 1;
    } else if (st.iters > 1 && corr > 0.5 * st.corr_prev) {
      st.status = (corr <= fmax(corr_tol, kStallTol)) ? 1 : 2;
    } else if (st.iters >= max_refine) {
      st.status = 2;
    }
    st.corr = corr;
    st.corr_prev = corr;
    state[s] = st;
    if (st.status == 0) atomicAdd(active, 1u);
  }
}

__global__ void batch_state_init_kernel(int count, const hp_batch_item *__restrict__ items,
                                        const int *__restrict__ info, BatchState *state, int refine) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= count) return;
  BatchState st;
  // a non-local system's refinement residual holds sqrt(w) of its mesh in LDS
  const bool too_fine = refine && items[s].sys.vnl && items[s].sys.nr > kNlMaxPoints;
  st.status = too_fine ? 4 : (info && info[s] != 0) ? 3 : (refine ? 0 : 1);
  st.iters = 0;
  st.corr_prev = 0.0;
  st.corr = 0.0;
  state[s] = st;
}

__global__ void batch_rmatrix_kernel(int count, const hp_batch_item *__restrict__ items,
                                     const cplx<double> *__restrict__ X, cplx<double> *__restrict__ R) {
  const int s = blockIdx.x;
  if (s >= count) return;
  const hp_batch_item it = items[s];
  const int nc = it.sys.nc, nr = it.sys.nr;
  const double f = it.sys.hbar2_2mu / it.sys.a;
  for (int e = threadIdx.x; e < nc * nc; e += 256) {
    const int c = e / nc, cp = e - c * nc;
    double re = 0.0, im = 0.0;
    for (int i = 0; i < nr; ++i) {
      const cplx<double> xv = X[it.x_off + (long)(c * nr + i) * nc + cp];
      re += it.sys.q[i] * xv.re;
      im += it.sys.q[i] * xv.im;
    }
    R[it.r_off + e] = cplx<double>{f * re, f * im};
  }
}

// ------------------------------------------------------- stepped solves --
// The solves of a bucket of larger systems, in steps of kSB rows: per step
// one launch of every system's diagonal block (one thread per right-hand
// column) and one launch of all update tiles of the rows beyond it (K = kSB).
constexpr int kSB = 64;

// P B (mode 0) or P R / s (mode 1, systems still refining) into Y.
template <typename T>
__global__ __launch_bounds__(256) void batch_rhs_kernel(int count, const hp_batch_item *__restrict__ items,
                                                        const int *__restrict__ perm, cplx<T> *__restrict__ Y,
                                                        const cplx<double> *__restrict__ Rr,
                                                        const double *__restrict__ cscale,
                                                        const BatchState *state, int mode) {
  const int s = blockIdx.x;
  if (s >= count) return;
  if (mode == 1 && state[s].status != 0) return;
  const hp_batch_item it = items[s];
  const int nc = it.sys.nc, nr = it.sys.nr, n = nc * nr;
  const int *pm = perm + it.p_off;
  cplx<T> *y = Y + it.x_off;
  for (long e = threadIdx.x; e < (long)n * nc; e += 256) {
    const int i = (int)(e / nc), cc = (int)(e - (long)i * nc);
    const int src = pm[i];
    cplx<T> v{T(0), T(0)};
    if (mode == 0) {
      const int c = src / nr, ii = src - c * nr;
      if (c == cc) v.re = (T)it.sys.q[ii];
    } else {
      const cplx<double> r = Rr[it.x_off + (long)src * nc + cc];
      const double sc = cscale[it.c_off + cc];
      v = cplx<T>{(T)(r.re / sc), (T)(r.im / sc)};
    }
    y[e] = v;
  }
}

template <typename T>
__global__ __launch_bounds__(256) void batch_widen_kernel(int count, const hp_batch_item *__restrict__ items,
                                                          const cplx<T> *__restrict__ Y, cplx<double> *__restrict__ X) {
  const int s = blockIdx.x;
  if (s >= count) return;
  const hp_batch_item it = items[s];
  const long cnt = (long)it.sys.nc * it.sys.nr * it.sys.nc;
  for (long e = threadIdx.x; e < cnt; e += 256)
    X[it.x_off + e] = cplx<double>{(double)Y[it.x_off + e].re, (double)Y[it.x_off + e].im};
}

// Tile offsets of every solve step (exclusive prefix sums, count + 1 per step):
// forward: the rows below the step's block; backward: the rows above it.
__global__ void batch_solve_tiles_kernel(int count, const hp_batch_item *__restrict__ items, int *fwd, int *bwd) {
  const int t = blockIdx.x;
  if (threadIdx.x != 0) return;
  const int b0 = t * kSB;
  int af = 0, ab = 0;
  int *of = fwd + (long)t * (count + 1), *ob = bwd + (long)t * (count + 1);
  for (int s = 0; s < count; ++s) {
    of[s] = af;
    ob[s] = ab;
    const int nc = items[s].sys.nc, n = item_n(items[s]);
    if (b0 < n) {
      const int below = n - b0 - min(kSB, n - b0);
      const int tn = (nc + 63) / 64;
      af += ((below + 63) / 64) * tn;
      ab += ((b0 + 63) / 64) * tn;
    }
  }
  of[count] = af;
  ob[count] = ab;
}

// Diagonal block [b0, b0 + bs) of every system (state: skip systems not
// refining): the block of LU staged in LDS, one right-hand column per thread
// (diag_block_solve).
// With STAGED the block's rows of Y (bs x nc) are first staged in LDS, so the
// substitution's reads of the rows solved before a group stay on chip (the
// same arithmetic as the unstaged form, which serves nc too large for LDS).
template <typename T, bool STAGED>
__global__ __launch_bounds__(256) void batch_sdiag_kernel(const hp_batch_item *__restrict__ items,
                                                          const cplx<T> *__restrict__ LU, cplx<T> *__restrict__ Y,
                                                          int b0, int upper, const BatchState *state) {
  // every lane reads the same element of D (a broadcast), so no padding
  __shared__ cplx<T> D[kSB * kSB];
  extern __shared__ __align__(16) char smem_raw[];
  cplx<T> *Ys = reinterpret_cast<cplx<T> *>(smem_raw);  // [bs][nc] (STAGED)
  const int s = blockIdx.x;
  if (state && state[s].status != 0) return;
  const hp_batch_item it = items[s];
  const int nc = it.sys.nc, n = item_n(it);
  if (b0 >= n) return;
  const int bs = min(kSB, n - b0);
  const cplx<T> *lu = LU + it.a_off;
  for (int e = threadIdx.x; e < kSB * kSB; e += blockDim.x) {
    const int r = e / kSB, k = e - r * kSB;
    D[e] = (r < bs && k < bs) ? lu[(long)(b0 + r) * n + b0 + k] : cplx<T>{T(0), T(0)};
  }
  cplx<T> *yb = Y + it.x_off + (long)b0 * nc;  // the block's rows
  if constexpr (STAGED) {
    for (int e = threadIdx.x; e < bs * nc; e += blockDim.x) Ys[e] = yb[e];
    __syncthreads();
    for (int c = threadIdx.x; c < nc; c += 256) diag_block_solve<T, kSB>(D, Ys, nc, 0, bs, c, upper != 0);
    __syncthreads();
    for (int e = threadIdx.x; e < bs * nc; e += blockDim.x) yb[e] = Ys[e];
  } else {
    __syncthreads();
    for (int c = threadIdx.x; c < nc; c += 256) diag_block_solve<T, kSB>(D, yb, nc, 0, bs, c, upper != 0);
  }
}

// Update tiles of a solve step: forward Y[b0+bs:n] -= L[b0+bs:n, b0:b0+bs] Y[b0:b0+bs],
// backward Y[0:b0] -= U[0:b0, b0:b0+bs] Y[b0:b0+bs].
template <typename T>
__global__ __launch_bounds__(256) void batch_strail_kernel(int count, const hp_batch_item *__restrict__ items,
                                                           const cplx<T> *__restrict__ LU, cplx<T> *__restrict__ Y,
                                                           const int *__restrict__ offs, int b0, int upper,
                                                           const BatchState *state) {
  extern __shared__ __align__(16) char smem_raw[];
  cplx<T> *As = reinterpret_cast<cplx<T> *>(smem_raw);
  cplx<T> *Bs = As + kBK * kBLd;
  const int g = blockIdx.x;
  if (g >= offs[count]) return;
  int lo = 0, hi = count;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (offs[mid] <= g)
      lo = mid;
    else
      hi = mid;
  }
  if (state && state[lo].status != 0) return;
  const hp_batch_item it = items[lo];
  const int nc = it.sys.nc, n = item_n(it);
  const int bs = min(kSB, n - b0);
  const int tn = (nc + 63) / 64;
  const int l = g - offs[lo];
  const cplx<T> *lu = LU + it.a_off;
  cplx<T> *y = Y + it.x_off;
  if (!upper)
    tile_gemm_sub<T>((l / tn) * 64, (l % tn) * 64, n - b0 - bs, nc, bs, lu + (long)(b0 + bs) * n + b0, n,
                     y + (long)b0 * nc, nc, y + (long)(b0 + bs) * nc, nc, As, Bs);
  else
    tile_gemm_sub<T>((l / tn) * 64, (l % tn) * 64, b0, nc, bs, lu + b0, n, y + (long)b0 * nc, nc, y, nc, As, Bs);
}

struct BatchWork {
  unsigned *counter;  // [2]: work queue, active count
  BatchState *state;  // [count]
  double *cscale;     // [sum nc]
  cplx<double> *res;  // [sum n nc] FP64 residual
  char *y;            // [sum n nc] working-precision right-hand sides
  int *fwd, *bwd;     // [steps][count + 1] tile offsets of the stepped solves
};

int solve_steps(int nmax) { return (nmax + kSB - 1) / kSB; }

BatchWork carve(char *w, int count, long sum_nc, long sum_xn, int prec) {
  const size_t elt = prec == HP_C64 ? sizeof(cplx<float>) : sizeof(cplx<double>);
  BatchWork b;
  size_t off = 0;
  b.counter = (unsigned *)(w + off);
  off += 256;
  b.state = (BatchState *)(w + off);
  off += align_up(sizeof(BatchState) * (size_t)count, 256);
  b.cscale = (double *)(w + off);
  off += align_up(sizeof(double) * (size_t)sum_nc, 256);
  b.res = (cplx<double> *)(w + off);
  off += align_up(sizeof(cplx<double>) * (size_t)sum_xn, 256);
  b.y = w + off;
  off += align_up(elt * (size_t)sum_xn, 256);
  b.fwd = (int *)(w + off);
  b.bwd = nullptr;
  return b;
}

size_t batch_bytes(int count, long sum_nc, long sum_xn, int nmax, int prec) {
  const size_t elt = prec == HP_C64 ? sizeof(cplx<float>) : sizeof(cplx<double>);
  return 256 + align_up(sizeof(BatchState) * (size_t)count, 256) + align_up(sizeof(double) * (size_t)sum_nc, 256) +
         align_up(sizeof(cplx<double>) * (size_t)sum_xn, 256) + align_up(elt * (size_t)sum_xn, 256) +
         align_up(sizeof(int) * 2 * (size_t)solve_steps(std::max(nmax, 1)) * (count + 1), 256) +
         align_up(sizeof(int) * 4 * (size_t)std::max(nmax, 1) * (count + 1), 256);  // stepped factor tables
}

// shape_host: HOST (n, nc) pairs of the systems, largest n first.
int check_shapes(int count, const int *shape_host, int *nmax) {
  *nmax = 0;
  for (int s = 0; s < count; ++s) {
    const int n = shape_host[2 * s], nc = shape_host[2 * s + 1];
    if (n < 1 || nc < 1 || (s > 0 && n > shape_host[2 * s - 2])) return HP_ERR_ARG;
    *nmax = std::max(*nmax, n);
  }
  return HP_OK;
}

// One stepped solve of every system (mode 0: of P B, then X = Y; mode 1: of
// the scaled residuals of the systems still refining).
template <typename T>
int stepped_solve(int count, const hp_batch_item *items, const int *shape_host, int nmax, const cplx<T> *LU,
                  const int *perm, cplx<T> *Y, cplx<double> *X, const BatchWork &w, int mode, hipStream_t st) {
  const int steps = solve_steps(nmax);
  const BatchState *state = mode == 1 ? w.state : nullptr;
  const int *fwd = w.fwd, *bwd = w.fwd + (long)steps * (count + 1);
  const size_t shm = tile_lds_bytes<T>();
  int rc;
  if ((rc = ensure_dynamic_lds((const void *)batch_strail_kernel<T>, shm))) return rc;
  // diagonal blocks with Y's block rows in LDS when every system's fit
  int ncmax = 1;
  for (int s = 0; s < count; ++s) ncmax = std::max(ncmax, shape_host[2 * s + 1]);
  const size_t yshm = (size_t)kSB * ncmax * sizeof(cplx<T>);
  const bool staged = yshm + sizeof(cplx<T>) * kSB * kSB <= 150 * 1024;
  if (staged && (rc = ensure_dynamic_lds((const void *)batch_sdiag_kernel<T, true>, yshm))) return rc;
  hipLaunchKernelGGL(batch_rhs_kernel<T>, dim3(count), dim3(256), 0, st, count, items, perm, Y,
                     (const cplx<double> *)w.res, (const double *)w.cscale, (const BatchState *)w.state, mode);
  HP_CHECK_LAUNCH();
  for (int pass = 0; pass < 2; ++pass) {
    const int upper = pass;
    for (int q = 0; q < steps; ++q) {
      const int t = upper ? steps - 1 - q : q;
      const int b0 = t * kSB;
      int active = 0;
      long tiles = 0;
      for (int s = 0; s < count && shape_host[2 * s] > b0; ++s) {
        ++active;
        const int n = shape_host[2 * s], nc = shape_host[2 * s + 1];
        const long rows = upper ? b0 : n - b0 - std::min(kSB, n - b0);
        tiles += ((rows + 63) / 64) * ((nc + 63) / 64);
      }
      if (staged)
        hipLaunchKernelGGL((batch_sdiag_kernel<T, true>), dim3(active), dim3(256), yshm, st, items, LU, Y, b0, upper,
                           state);
      else
        hipLaunchKernelGGL((batch_sdiag_kernel<T, false>), dim3(active), dim3(256), 0, st, items, LU, Y, b0, upper,
                           state);
      HP_CHECK_LAUNCH();
      if (tiles == 0) continue;
      hipLaunchKernelGGL(batch_strail_kernel<T>, dim3((unsigned)tiles), dim3(256), shm, st, active, items, LU, Y,
                         (upper ? bwd : fwd) + (long)t * (count + 1), b0, upper, state);
      HP_CHECK_LAUNCH();
    }
  }
  if (X) {
    hipLaunchKernelGGL(batch_widen_kernel<T>, dim3(count), dim3(256), 0, st, count, items, Y, X);
    HP_CHECK_LAUNCH();
  }
  return HP_OK;
}

}  // namespace

}  // namespace hp

using namespace hp;

extern "C" size_t hp_batch_workspace_bytes(int count, long sum_nc, long sum_xn, int nmax, int prec) {
  if (count < 1 || sum_nc < 1 || sum_xn < 1 || nmax < 1 || (prec != HP_C64 && prec != HP_C128)) return 0;
  return batch_bytes(count, sum_nc, sum_xn, nmax, prec);
}

extern "C" int hp_batch_build(int count, const hp_batch_item *items, int prec, void *A, void *stream) {
  if (count < 1 || !items || !A) return HP_ERR_ARG;
  hipStream_t st = (hipStream_t)stream;
  TraceScope ts(TR_ASSEMBLE, st, 0.0, 0.0);
  if (count > 65535) return HP_ERR_UNSUPPORTED;  // grid y limit
  if (prec == HP_C64)
    hipLaunchKernelGGL(batch_build_kernel<float>, dim3(kBuildGroups, count), dim3(256), 0, st, count, items,
                       (cplx<float> *)A);
  else if (prec == HP_C128)
    hipLaunchKernelGGL(batch_build_kernel<double>, dim3(kBuildGroups, count), dim3(256), 0, st, count, items,
                       (cplx<double> *)A);
  else
    return HP_ERR_ARG;
  HP_CHECK_LAUNCH();
  return HP_OK;
}

extern "C" int hp_batch_factor(int count, const hp_batch_item *items, int prec, void *A, int *ipiv, int *perm,
                               int *info, int panel, int groups, void *work, size_t work_bytes, void *stream) {
  if (count < 1 || !items || !A || !ipiv || !perm || !info || !work || work_bytes < 256) return HP_ERR_ARG;
  if (panel < 1 || panel > kBK || groups < 1) return HP_ERR_ARG;
  if (prec != HP_C64 && prec != HP_C128) return HP_ERR_ARG;
  hipStream_t st = (hipStream_t)stream;
  unsigned *counter = (unsigned *)work;
  hipLaunchKernelGGL(batch_zero_kernel, dim3(1), dim3(64), 0, st, counter, 2);
  HP_CHECK_LAUNCH();
  const int grid = std::min(count, groups);
  TraceScope ts(TR_PANEL, st, 0.0, 0.0);
  int rc;
  if (prec == HP_C64) {
    const size_t shm = tile_lds_bytes<float>();
    if ((rc = ensure_dynamic_lds((const void *)batch_lu_kernel<float>, shm))) return rc;
    hipLaunchKernelGGL(batch_lu_kernel<float>, dim3(grid), dim3(256), shm, st, count, items, (cplx<float> *)A, ipiv,
                       perm, info, counter, panel);
  } else {
    const size_t shm = tile_lds_bytes<double>();
    if ((rc = ensure_dynamic_lds((const void *)batch_lu_kernel<double>, shm))) return rc;
    hipLaunchKernelGGL(batch_lu_kernel<double>, dim3(grid), dim3(256), shm, st, count, items, (cplx<double> *)A,
                       ipiv, perm, info, counter, panel);
  }
  HP_CHECK_LAUNCH();
  return HP_OK;
}

extern "C" int hp_batch_factor_stepped(int count, const hp_batch_item *items, const int *n_host, int prec,
                                       void *A, int *ipiv, int *perm, int *info, int panel, int block, void *work,
                                       size_t work_bytes, void *stream) {
  if (count < 1 || !items || !n_host || !A || !ipiv || !perm || !info || !work) return HP_ERR_ARG;
  if (panel < 1 || panel > kBK || (prec != HP_C64 && prec != HP_C128)) return HP_ERR_ARG;
  if (block < panel || block > kBlockMax || block % panel != 0) return HP_ERR_ARG;
  int nmax = 0;
  for (int s = 0; s < count; ++s) {
    if (n_host[s] < 1 || (s > 0 && n_host[s] > n_host[s - 1])) return HP_ERR_ARG;  // largest first
    nmax = std::max(nmax, n_host[s]);
  }
  const int P = (nmax + panel - 1) / panel;     // panel steps
  const int NBk = (nmax + block - 1) / block;  // outer blocks
  const int Q = 2 * P + 2 * NBk;
  const size_t tbl = 256 + sizeof(int) * (size_t)Q * (count + 1);
  if (work_bytes < tbl) return HP_ERR_WORKSPACE;
  int *offs = (int *)((char *)work + 256);
  hipStream_t st = (hipStream_t)stream;
  hipLaunchKernelGGL(batch_zero_kernel, dim3((count + 255) / 256), dim3(256), 0, st, (unsigned *)info, count);
  HP_CHECK_LAUNCH();
  hipLaunchKernelGGL(batch_tables_kernel, dim3(Q), dim3(64), 0, st, count, items, panel, block, P, offs);
  HP_CHECK_LAUNCH();
  // FP64 trailing tiles: the direct-staged tile product (32 KB of LDS)
  const size_t shm = prec == HP_C64 ? tile_lds_bytes<float>() : kDirect64TileLds;
  int rc = prec == HP_C64 ? ensure_dynamic_lds((const void *)batch_trail_kernel<float>, shm)
                          : ensure_dynamic_lds((const void *)batch_trail_kernel<double>, shm);
  if (rc) return rc;
  // units of one tiled step over the systems still factoring (host count,
  // the same formula as the device tables)
  auto units = [&](int kind, int j, int *active) {
    long u = 0;
    int a = 0;
    for (int s = 0; s < count && n_host[s] > j; ++s) {
      ++a;
      u += step_units(kind, n_host[s], j, panel, block);
    }
    *active = a;
    return u;
  };
  TraceScope ts(TR_PANEL, st, 0.0, 0.0);
  for (int J = 0; J < nmax; J += block) {
    for (int j0 = J; j0 < std::min(J + block, nmax); j0 += panel) {
      int active = 0;
      const long tiles = units(0, j0, &active);
      // FP32 panels of 8 columns on at most 4096 rows: held in registers
      const int prows = n_host[0] - j0;
      if (prec == HP_C64 && panel == 8 && prows <= 4 * kRegPanelThreads && g_reg_panel.load() != 0) {
        if (prows <= kRegPanelThreads)
          hipLaunchKernelGGL((batch_panel_reg_kernel<float, 8, 1>), dim3(active), dim3(kRegPanelThreads), 0, st, items,
                             (cplx<float> *)A, ipiv, perm, info, j0);
        else if (prows <= 2 * kRegPanelThreads)
          hipLaunchKernelGGL((batch_panel_reg_kernel<float, 8, 2>), dim3(active), dim3(kRegPanelThreads), 0, st, items,
                             (cplx<float> *)A, ipiv, perm, info, j0);
        else
          hipLaunchKernelGGL((batch_panel_reg_kernel<float, 8, 4>), dim3(active), dim3(kRegPanelThreads), 0, st, items,
                             (cplx<float> *)A, ipiv, perm, info, j0);
      } else if (prec == HP_C64)
        hipLaunchKernelGGL(batch_panel_kernel<float>, dim3(active), dim3(256), 0, st, items, (cplx<float> *)A, ipiv,
                           perm, info, j0, panel, block);
      else
        hipLaunchKernelGGL(batch_panel_kernel<double>, dim3(active), dim3(256), 0, st, items, (cplx<double> *)A,
                           ipiv, perm, info, j0, panel, block);
      HP_CHECK_LAUNCH();
      {
        int act3 = 0;
        const long chunks = units(3, j0, &act3);
        const int *o3 = offs + (long)(P + j0 / panel) * (count + 1);
        if (chunks > 0) {
          if (prec == HP_C64)
            hipLaunchKernelGGL(batch_swap_brow_kernel<float>, dim3((unsigned)chunks), dim3(256), 0, st, act3, items,
                               (cplx<float> *)A, ipiv, o3, j0, panel, block);
          else
            hipLaunchKernelGGL(batch_swap_brow_kernel<double>, dim3((unsigned)chunks), dim3(256), 0, st, act3, items,
                               (cplx<double> *)A, ipiv, o3, j0, panel, block);
          HP_CHECK_LAUNCH();
        }
      }
      if (tiles == 0) continue;
      if (tiles > (1L << 30)) return HP_ERR_UNSUPPORTED;
      const int *o = offs + (long)(j0 / panel) * (count + 1);
      if (prec == HP_C64)
        hipLaunchKernelGGL(batch_trail_kernel<float>, dim3((unsigned)tiles), dim3(256), shm, st, active, items,
                           (cplx<float> *)A, o, 0, j0, panel, block);
      else
        hipLaunchKernelGGL(batch_trail_kernel<double>, dim3((unsigned)tiles), dim3(256), shm, st, active, items,
                           (cplx<double> *)A, o, 0, j0, panel, block);
      HP_CHECK_LAUNCH();
    }
    int active = 0;
    const long chunks = units(2, J, &active);
    if (chunks == 0) continue;
    const long tiles = units(1, J, &active);
    if (tiles > (1L << 30)) return HP_ERR_UNSUPPORTED;
    const int qb = 2 * P + 2 * (J / block);
    const int *ob = offs + (long)qb * (count + 1), *ou = offs + (long)(qb + 1) * (count + 1);
    if (prec == HP_C64) {
      hipLaunchKernelGGL(batch_brow_kernel<float>, dim3((unsigned)chunks), dim3(256), 0, st, active, items,
                         (cplx<float> *)A, ob, J, block);
      HP_CHECK_LAUNCH();
      hipLaunchKernelGGL(batch_trail_kernel<float>, dim3((unsigned)tiles), dim3(256), shm, st, active, items,
                         (cplx<float> *)A, ou, 1, J, panel, block);
    } else {
      hipLaunchKernelGGL(batch_brow_kernel<double>, dim3((unsigned)chunks), dim3(256), 0, st, active, items,
                         (cplx<double> *)A, ob, J, block);
      HP_CHECK_LAUNCH();
      hipLaunchKernelGGL(batch_trail_kernel<double>, dim3((unsigned)tiles), dim3(256), shm, st, active, items,
                         (cplx<double> *)A, ou, 1, J, panel, block);
    }
    HP_CHECK_LAUNCH();
  }
  return HP_OK;
}

extern "C" int hp_batch_solve_init(int count, const hp_batch_item *items, const int *shape_host, int prec,
                                   const void *LU, const int *perm, const int *info_factor, double *X, int refine,
                                   long sum_nc, long sum_xn, void *work, size_t work_bytes, void *stream) {
  if (count < 1 || !items || !LU || !perm || !X || !work) return HP_ERR_ARG;
  if (prec != HP_C64 && prec != HP_C128) return HP_ERR_ARG;
  int nmax = 1, rc;
  if (shape_host && (rc = check_shapes(count, shape_host, &nmax))) return rc;
  if (work_bytes < batch_bytes(count, sum_nc, sum_xn, nmax, prec)) return HP_ERR_WORKSPACE;
  hipStream_t st = (hipStream_t)stream;
  BatchWork w = carve((char *)work, count, sum_nc, sum_xn, prec);
  hipLaunchKernelGGL(batch_state_init_kernel, dim3((count + 255) / 256), dim3(256), 0, st, count, items,
                     info_factor, w.state, refine);
  HP_CHECK_LAUNCH();
  TraceScope ts(TR_TRSM, st, 0.0, 0.0);
  if (shape_host) {
    const int steps = solve_steps(nmax);
    hipLaunchKernelGGL(batch_solve_tiles_kernel, dim3(steps), dim3(64), 0, st, count, items, w.fwd,
                       w.fwd + (long)steps * (count + 1));
    HP_CHECK_LAUNCH();
    if (prec == HP_C64)
      return stepped_solve<float>(count, items, shape_host, nmax, (const cplx<float> *)LU, perm, (cplx<float> *)w.y,
                                  (cplx<double> *)X, w, 0, st);
    return stepped_solve<double>(count, items, shape_host, nmax, (const cplx<double> *)LU, perm,
                                 (cplx<double> *)X, nullptr, w, 0, st);
  }
  if (prec == HP_C64) {
    const size_t shm = tile_lds_bytes<float>();
    if ((rc = ensure_dynamic_lds((const void *)batch_solve_kernel<float>, shm))) return rc;
    hipLaunchKernelGGL(batch_solve_kernel<float>, dim3(count), dim3(256), shm, st, count, items,
                       (const cplx<float> *)LU, perm, (cplx<float> *)w.y, (cplx<double> *)X,
                       (const cplx<double> *)nullptr, (const double *)nullptr, w.state, 0);
  } else {
    const size_t shm = tile_lds_bytes<double>();
    if ((rc = ensure_dynamic_lds((const void *)batch_solve_kernel<double>, shm))) return rc;
    hipLaunchKernelGGL(batch_solve_kernel<double>, dim3(count), dim3(256), shm, st, count, items,
                       (const cplx<double> *)LU, perm, (cplx<double> *)X, (cplx<double> *)nullptr,
                       (const cplx<double> *)nullptr, (const double *)nullptr, w.state, 0);
  }
  HP_CHECK_LAUNCH();
  return HP_OK;
}

extern "C" int hp_batch_refine_step(int count, const hp_batch_item *items, const int *shape_host, const void *LU,
                                    const int *perm, double *X, int max_refine, double tol, long sum_nc,
                                    long sum_xn, void *work, size_t work_bytes, void *stream) {
  if (count < 1 || !items || !LU || !perm || !X || !work) return HP_ERR_ARG;
  int nmax = 1, rc;
  if (shape_host && (rc = check_shapes(count, shape_host, &nmax))) return rc;
  if (work_bytes < batch_bytes(count, sum_nc, sum_xn, nmax, HP_C64)) return HP_ERR_WORKSPACE;
  hipStream_t st = (hipStream_t)stream;
  BatchWork w = carve((char *)work, count, sum_nc, sum_xn, HP_C64);
  hipLaunchKernelGGL(batch_zero_kernel, dim3(1), dim3(64), 0, st, w.counter + 1, 1);
  HP_CHECK_LAUNCH();
  {
    TraceScope ts(TR_RESIDUAL, st, 0.0, 0.0);
    hipLaunchKernelGGL(batch_res_kinetic_kernel, dim3(kResChunks, count), dim3(256), 0, st, count, items,
                       (const cplx<double> *)X, w.res, w.cscale, w.state);
    HP_CHECK_LAUNCH();
    hipLaunchKernelGGL(batch_res_nonlocal_kernel, dim3(kResChunks, count), dim3(256), 0, st, count, items,
                       (const cplx<double> *)X, w.res, w.state);
    HP_CHECK_LAUNCH();
    hipLaunchKernelGGL(batch_res_coupling_kernel, dim3(kResChunks, count), dim3(256), 0, st, count, items,
                       (const cplx<double> *)X, w.res, w.cscale, w.state);
    HP_CHECK_LAUNCH();
    hipLaunchKernelGGL(batch_res_scale_kernel, dim3(count), dim3(64), 0, st, count, items, w.cscale, w.state);
    HP_CHECK_LAUNCH();
  }
  {
    TraceScope ts(TR_TRSM, st, 0.0, 0.0);
    if (shape_host) {
      if ((rc = stepped_solve<float>(count, items, shape_host, nmax, (const cplx<float> *)LU, perm,
                                     (cplx<float> *)w.y, nullptr, w, 1, st)))
        return rc;
    } else {
      const size_t shm = tile_lds_bytes<float>();
      if ((rc = ensure_dynamic_lds((const void *)batch_solve_kernel<float>, shm))) return rc;
      hipLaunchKernelGGL(batch_solve_kernel<float>, dim3(count), dim3(256), shm, st, count, items,
                         (const cplx<float> *)LU, perm, (cplx<float> *)w.y, (cplx<double> *)nullptr, w.res,
                         w.cscale, w.state, 1);
      HP_CHECK_LAUNCH();
    }
  }
  TraceScope ts(TR_REFINE, st, 0.0, 0.0);
  hipLaunchKernelGGL(batch_update_kernel<float>, dim3(count), dim3(256), 0, st, count, items,
                     (const cplx<float> *)w.y, (cplx<double> *)X, w.cscale, w.state, tol, max_refine,
                     w.counter + 1);
  HP_CHECK_LAUNCH();
  return HP_OK;
}

extern "C" int hp_set_batch_reg_panel(int on) { return g_reg_panel.exchange(on ? 1 : 0); }

extern "C" int hp_batch_active(const void *work, unsigned *active, void *stream) {
  if (!work || !active) return HP_ERR_ARG;
  hipStream_t st = (hipStream_t)stream;
  HP_CHECK_HIP(hipMemcpyAsync(active, (const unsigned *)work + 1, sizeof(unsigned), hipMemcpyDeviceToHost, st));
  HP_CHECK_HIP(hipStreamSynchronize(st));
  return HP_OK;
}

extern "C" int hp_batch_status(int count, const void *work, int *status, int *iters, void *stream) {
  if (count < 1 || !work || !status) return HP_ERR_ARG;
  hipStream_t st = (hipStream_t)stream;
  // the state array follows the 256-byte counter block
  std::vector<BatchState> host((size_t)count);
  HP_CHECK_HIP(hipMemcpyAsync(host.data(), (const char *)work + 256, sizeof(BatchState) * (size_t)count,
                              hipMemcpyDeviceToHost, st));
  HP_CHECK_HIP(hipStreamSynchronize(st));
  for (int s = 0; s < count; ++s) {
    status[s] = host[(size_t)s].status;
    if (iters) iters[s] = host[(size_t)s].iters;
  }
  return HP_OK;
}

extern "C" int hp_batch_rmatrix(int count, const hp_batch_item *items, const double *X, double *R, void *stream) {
  if (count < 1 || !items || !X || !R) return HP_ERR_ARG;
  hipStream_t st = (hipStream_t)stream;
  TraceScope ts(TR_RMATRIX, st, 0.0, 0.0);
  hipLaunchKernelGGL(batch_rmatrix_kernel, dim3(count), dim3(256), 0, st, count, items, (const cplx<double> *)X,
                     (cplx<double> *)R);
  HP_CHECK_LAUNCH();
  return HP_OK;
}

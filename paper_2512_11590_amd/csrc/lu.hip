// Blocked right-looking complex LU with partial pivoting, and the triangular
// solves that use its factors (Sec. 3.1: M = P L U, then forward and backward
// substitution; Sec. 3.4: the same in FP32).
//
// Storage: row-major, interleaved complex, leading dimension lda.  Row
// interchanges therefore move contiguous memory, and since the system matrix
// is complex symmetric the row-major array is also its column-major array.
//
// Structure of hp_factor for an outer block of kOuterBlock columns at k:
//   for each inner panel of kPanelWidth columns j inside the block:
//     panel_kernel       cooperative grid, one grid barrier per column: pivot
//                        search (wavefront shuffles + slot exchange), row swap,
//                        scaling and rank-1 update of the panel held in LDS
//     laswp_kernel       the panel's swaps on the other columns of the block
//     trsm + gemm_sub    U rows of the panel and update of the rest of the block
//   laswp_kernel         the block's swaps on every column outside the block
//   trsm_lower_unit      U12 = L11^-1 A12
//   gemm_sub             A22 -= L21 U12 (MFMA complex GEMM, 4 real products)
#include "common.h"

#include <algorithm>
#include <climits>

namespace hp {

// ------------------------------------------------------------------ utils --

__global__ void fill_u32_kernel(unsigned *p, size_t n, unsigned v) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

static int fill_u32(unsigned *p, size_t n, unsigned v, hipStream_t st) {
  if (n == 0) return HP_OK;
  hipLaunchKernelGGL(fill_u32_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, n, v);
  HP_CHECK_LAUNCH();
  return HP_OK;
}

template <typename T>
__device__ __forceinline__ void argmax_combine(T &v, int &r, T ov, int orow) {
  if (ov > v || (ov == v && orow < r)) {
    v = ov;
    r = orow;
  }
}

// Data exchanged between workgroups of one grid goes through agent-scope
// atomic loads and stores, which are coherent across the chip's XCDs.
__device__ __forceinline__ void st_agent(double *p, double v) {
  __hip_atomic_store(reinterpret_cast<unsigned long long *>(p), __double_as_longlong(v), __ATOMIC_RELAXED,
                     __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double ld_agent(const double *p) {
  return __longlong_as_double(__hip_atomic_load(reinterpret_cast<const unsigned long long *>(p), __ATOMIC_RELAXED,
                                                __HIP_MEMORY_SCOPE_AGENT));
}
__device__ __forceinline__ void st_agent(float *p, float v) {
  __hip_atomic_store(reinterpret_cast<unsigned *>(p), __float_as_uint(v), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ float ld_agent(const float *p) {
  return __uint_as_float(
      __hip_atomic_load(reinterpret_cast<const unsigned *>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
}
__device__ __forceinline__ void st_agent(int *p, int v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int ld_agent(const int *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ void st_agent(cplx<T> *p, cplx<T> v) {
  st_agent(&p->re, v.re);
  st_agent(&p->im, v.im);
}
template <typename T>
__device__ __forceinline__ cplx<T> ld_agent(const cplx<T> *p) {
  return cplx<T>{ld_agent(&p->re), ld_agent(&p->im)};
}

// (value, row) argmax over the 64 lanes of a wavefront; ties -> smaller row.
template <typename T>
__device__ __forceinline__ void wave_argmax(T &v, int &r) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    T ov = __shfl_xor(v, off);
    int orow = __shfl_xor(r, off);
    argmax_combine(v, r, ov, orow);
  }
}

// Whole-workgroup argmax (256 threads); every thread returns the result.
template <typename T>
__device__ __forceinline__ void block_argmax(T &v, int &r, T *sv, int *sr) {
  wave_argmax(v, r);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  __syncthreads();
  if (lane == 0) {
    sv[wave] = v;
    sr[wave] = r;
  }
  __syncthreads();
  v = sv[0];
  r = sr[0];
#pragma unroll
  for (int w = 1; w < 4; ++w) argmax_combine(v, r, sv[w], sr[w]);
}

// Two-level grid barrier for a cooperative launch.  Workgroups arrive on one
// of several group counters (spread over separate cache lines), the last
// arrival of each group bumps the top counter, and everyone waits on the top
// counter.  The wait is bounded: on expiry it records -1 in *flag and stops
// waiting, and later barriers return at once, so the grid always drains.
constexpr int kBarGroup = 16;     // workgroups per group counter
constexpr int kBarStride = 32;    // unsigned words between counters (128 B)

__device__ __forceinline__ void grid_barrier(unsigned *bar, unsigned ngroups, unsigned epoch,
                                             int *flag) {
  // every lane's agent-scope stores must have completed before the arrival
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned g = blockIdx.x / kBarGroup;
    const unsigned gsize = min((unsigned)kBarGroup, gridDim.x - g * kBarGroup);
    unsigned *top = bar;
    unsigned *grp = bar + (g + 1) * kBarStride;
    unsigned old = atomicAdd(grp, 1u);
    if (old + 1 == gsize * epoch) atomicAdd(top, 1u);
    unsigned spins = 0;
    while (__hip_atomic_load(top, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < ngroups * epoch) {
      __builtin_amdgcn_s_sleep(1);
      if (((++spins) & 1023u) == 0) {
        if (spins > kSpinLimit ||
            __hip_atomic_load(flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == -1) {
          atomicExch(flag, -1);
          break;
        }
      }
    }
  }
  __syncthreads();
}

static size_t barrier_words(int G) { return (size_t)(((G + kBarGroup - 1) / kBarGroup) + 1) * kBarStride; }

// ------------------------------------------------------------ panel (LU) --
//
// Factor columns [j0, j0+w) of rows [j0, n) with partial pivoting.  The rows
// are split into contiguous chunks of rpw rows, one per workgroup, held in
// LDS for the whole panel.  Per column: each workgroup finds its candidate
// pivot (largest |Re|+|Im|, smallest row on ties) and publishes it, with the
// candidate's full panel row, in a slot; the owner of the diagonal row
// publishes that row too; one grid barrier; every workgroup then picks the
// same winner from the slots, the owners of the two rows exchange them, and
// each workgroup scales and updates its own rows.  Slots alternate between
// two buffers so a slow reader never sees the next column's writes.
template <typename T>
__global__ __launch_bounds__(256) void panel_kernel(int n, int j0, int w, cplx<T> *__restrict__ A,
                                                    long lda, int *__restrict__ ipiv,
                                                    int *__restrict__ info, unsigned *bar,
                                                    cplx<T> *slot_rows, T *slot_val, int *slot_row,
                                                    cplx<T> *diag_rows, int rpw) {
  extern __shared__ __align__(16) char smem_raw[];
  cplx<T> *Ls = reinterpret_cast<cplx<T> *>(smem_raw);  // [rpw][kPanelWidth]
  __shared__ cplx<T> urow[kPanelWidth], drow[kPanelWidth];
  __shared__ T red_v[4];
  __shared__ int red_r[4];
  constexpr int W = kPanelWidth;
  const int G = gridDim.x, g = blockIdx.x, tid = threadIdx.x;
  const unsigned ngroups = (G + kBarGroup - 1) / kBarGroup;
  const int rbeg = j0 + g * rpw;
  const int rend = min(n, rbeg + rpw);
  const int nrow = max(0, rend - rbeg);

  for (int e = tid; e < nrow * w; e += 256) {
    const int rr = e / w, cc = e - rr * w;
    Ls[rr * W + cc] = A[(long)(rbeg + rr) * lda + j0 + cc];
  }
  __syncthreads();

  for (int j = 0; j < w; ++j) {
    const int jc = j0 + j;
    const int par = j & 1;
    // -- local pivot candidate in column j among rows >= jc
    T best = T(-1);
    int brow = INT_MAX;
    for (int rr = tid; rr < nrow; rr += 256) {
      const int gr = rbeg + rr;
      if (gr >= jc) argmax_combine(best, brow, cabs1(Ls[rr * W + j]), gr);
    }
    block_argmax(best, brow, red_v, red_r);
    if (tid == 0) {
      st_agent(&slot_val[par * G + g], best);
      st_agent(&slot_row[par * G + g], brow);
    }
    if (brow != INT_MAX)
      for (int cc = tid; cc < w; cc += 256)
        st_agent(&slot_rows[((size_t)par * G + g) * W + cc], Ls[(brow - rbeg) * W + cc]);
    if (jc >= rbeg && jc < rend)
      for (int cc = tid; cc < w; cc += 256) st_agent(&diag_rows[par * W + cc], Ls[(jc - rbeg) * W + cc]);
    grid_barrier(bar, ngroups, (unsigned)(j + 1), info);
    // -- global winner (identical in every workgroup)
    T wv = T(-1);
    int wr = INT_MAX;
    for (int e = tid; e < G; e += 256) argmax_combine(wv, wr, ld_agent(&slot_val[par * G + e]), ld_agent(&slot_row[par * G + e]));
    block_argmax(wv, wr, red_v, red_r);
    int p = wr;
    if (p < jc || p >= n) {  // cannot happen unless the exchange failed; never index out of range
      if (g == 0 && tid == 0) atomicExch(info, -1);
      p = jc;
    }
    // the winning row's values sit in the slot of the workgroup that owns row p
    const int wg = min(G - 1, (p - j0) / rpw);
    for (int cc = tid; cc < w; cc += 256) {
      urow[cc] = ld_agent(&slot_rows[((size_t)par * G + wg) * W + cc]);
      drow[cc] = ld_agent(&diag_rows[par * W + cc]);
    }
    __syncthreads();
    if (g == 0 && tid == 0) {
      ipiv[jc] = p;
      if (!(wv > T(0))) atomicCAS(info, 0, jc + 1);
    }
    if (jc >= rbeg && jc < rend)
      for (int cc = tid; cc < w; cc += 256) Ls[(jc - rbeg) * W + cc] = urow[cc];
    if (p != jc && p >= rbeg && p < rend)
      for (int cc = tid; cc < w; cc += 256) Ls[(p - rbeg) * W + cc] = drow[cc];
    __syncthreads();
    // -- scale the column below the pivot and update the rest of the panel
    const cplx<T> piv = urow[j];
    if (wv > T(0)) {
      const cplx<T> inv = crcp(piv);
      for (int rr = tid; rr < nrow; rr += 256) {
        const int gr = rbeg + rr;
        if (gr > jc) {
          const cplx<T> lv = cmul(Ls[rr * W + j], inv);
          Ls[rr * W + j] = lv;
          for (int cc = j + 1; cc < w; ++cc) Ls[rr * W + cc] = cfms(Ls[rr * W + cc], lv, urow[cc]);
        }
      }
    }
    __syncthreads();
  }
  for (int e = tid; e < nrow * w; e += 256) {
    const int rr = e / w, cc = e - rr * w;
    A[(long)(rbeg + rr) * lda + j0 + cc] = Ls[rr * W + cc];
  }
}

// ------------------------------------------------------------------ laswp --
//
// Apply the interchanges ipiv[k0..k1) in order to columns [c0, c1) and
// [c2, c3).  One lane per column; rows are contiguous, so each swap is a
// coalesced pair of row segments.  If perm is given, thread 0 of block 0
// applies the same interchanges to it.
template <typename T>
__global__ __launch_bounds__(256) void laswp_kernel(cplx<T> *__restrict__ A, long lda, const int *__restrict__ ipiv,
                                                    int k0, int k1, int c0, int c1, int c2, int c3,
                                                    int *__restrict__ perm) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const int n1 = c1 - c0;
  const int ntot = n1 + (c3 - c2);
  if (perm && t == 0) {
    for (int k = k0; k < k1; ++k) {
      const int p = ipiv[k];
      if (p != k) {
        int tmp = perm[k];
        perm[k] = perm[p];
        perm[p] = tmp;
      }
    }
  }
  if (t >= ntot) return;
  const int col = (t < n1) ? (int)(c0 + t) : (int)(c2 + (t - n1));
  for (int k = k0; k < k1; ++k) {
    const int p = ipiv[k];
    if (p != k) {
      cplx<T> a = A[(long)k * lda + col];
      cplx<T> b = A[(long)p * lda + col];
      A[(long)k * lda + col] = b;
      A[(long)p * lda + col] = a;
    }
  }
}

template <typename T>
static int laswp(cplx<T> *A, long lda, const int *ipiv, int k0, int k1, int c0, int c1, int c2, int c3,
                 int *perm, hipStream_t st) {
  const long ntot = (long)std::max(0, c1 - c0) + std::max(0, c3 - c2);
  if (k1 <= k0 || (ntot == 0 && !perm)) return HP_OK;
  const unsigned blocks = (unsigned)std::max<long>(1, (ntot + 255) / 256);
  TraceScope ts(TR_LASWP, st, 0.0, 4.0 * (k1 - k0) * ntot * sizeof(cplx<T>));
  hipLaunchKernelGGL(laswp_kernel<T>, dim3(blocks), dim3(256), 0, st, A, lda, ipiv, k0, k1, c0,
                     std::max(c0, c1), c2, std::max(c2, c3), perm);
  HP_CHECK_LAUNCH();
  return HP_OK;
}

__global__ void iota_kernel(int *p, int n) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = i;
}

// ------------------------------------------------------------------- trsm --
//
// X = L^-1 X (L unit lower, m x m) or X = U^-1 X (U upper, non-unit), X of
// m rows and ncols columns.  One workgroup per stripe of CW columns; the
// stripe lives in LDS.  Blocked by 16 rows: a 16 x 16 diagonal solve, then
// the rows below (above) are updated with the 16 solved rows.
template <typename T>
struct TrsmCfg {
  static constexpr int CW = 16;
};
template <>
struct TrsmCfg<float> {
  static constexpr int CW = 32;
};
constexpr int kTrsmMaxRows = 256;
constexpr int kTrsmBS = 16;

template <typename T, bool UPPER>
__global__ __launch_bounds__(256) void trsm_kernel(int m, int ncols, const cplx<T> *__restrict__ L, long ldl,
                                                   cplx<T> *__restrict__ X, long ldx) {
  constexpr int CW = TrsmCfg<T>::CW;
  constexpr int BS = kTrsmBS;
  extern __shared__ __align__(16) char smem_raw[];
  cplx<T> *Xs = reinterpret_cast<cplx<T> *>(smem_raw);  // [m][CW]
  __shared__ cplx<T> Ld[BS][BS + 1];
  const int tid = threadIdx.x;
  const int col0 = blockIdx.x * CW;
  const int ncw = min(CW, ncols - col0);
  for (int e = tid; e < m * CW; e += 256) {
    const int rr = e / CW, cc = e - rr * CW;
    Xs[e] = (cc < ncw) ? X[(long)rr * ldx + col0 + cc] : cplx<T>{T(0), T(0)};
  }
  __syncthreads();
  const int nblk = (m + BS - 1) / BS;
  for (int bi = 0; bi < nblk; ++bi) {
    const int b = UPPER ? (nblk - 1 - bi) : bi;
    const int r0 = b * BS;
    const int bs = min(BS, m - r0);
    // diagonal block into LDS (for UPPER store reciprocal of the diagonal)
    for (int e = tid; e < BS * BS; e += 256) {
      const int ii = e / BS, jj = e - ii * BS;
      cplx<T> v{T(0), T(0)};
      if (ii < bs && jj < bs) v = L[(long)(r0 + ii) * ldl + r0 + jj];
      if (UPPER && ii == jj && ii < bs) v = crcp(v);
      Ld[ii][jj] = v;
    }
    __syncthreads();
    // diagonal solve: CW threads, one per column
    if (tid < CW) {
      const int cc = tid;
      if (!UPPER) {
        for (int ii = 1; ii < bs; ++ii) {
          cplx<T> s = Xs[(r0 + ii) * CW + cc];
          for (int jj = 0; jj < ii; ++jj) s = cfms(s, Ld[ii][jj], Xs[(r0 + jj) * CW + cc]);
          Xs[(r0 + ii) * CW + cc] = s;
        }
      } else {
        for (int ii = bs - 1; ii >= 0; --ii) {
          cplx<T> s = Xs[(r0 + ii) * CW + cc];
          for (int jj = ii + 1; jj < bs; ++jj) s = cfms(s, Ld[ii][jj], Xs[(r0 + jj) * CW + cc]);
          Xs[(r0 + ii) * CW + cc] = cmul(s, Ld[ii][ii]);
        }
      }
    }
    __syncthreads();
    // update the remaining rows with the solved block
    const int ur0 = UPPER ? 0 : r0 + bs;
    const int ur1 = UPPER ? r0 : m;
    const int nu = ur1 - ur0;
    for (int e = tid; e < nu * CW; e += 256) {
      const int rr = ur0 + e / CW, cc = e % CW;
      cplx<T> s = Xs[rr * CW + cc];
      const cplx<T> *lrow = L + (long)rr * ldl + r0;
      for (int jj = 0; jj < bs; ++jj) s = cfms(s, lrow[jj], Xs[(r0 + jj) * CW + cc]);
      Xs[rr * CW + cc] = s;
    }
    __syncthreads();
  }
  for (int e = tid; e < m * CW; e += 256) {
    const int rr = e / CW, cc = e - rr * CW;
    if (cc < ncw) X[(long)rr * ldx + col0 + cc] = Xs[e];
  }
}

template <typename T, bool UPPER>
static int trsm(int m, int ncols, const cplx<T> *L, long ldl, cplx<T> *X, long ldx, hipStream_t st) {
  if (m <= 0 || ncols <= 0) return HP_OK;
  if (m > kTrsmMaxRows) return HP_ERR_ARG;
  constexpr int CW = TrsmCfg<T>::CW;
  const size_t shm = (size_t)m * CW * sizeof(cplx<T>);
  int rc = ensure_dynamic_lds((const void *)trsm_kernel<T, UPPER>, shm);
  if (rc) return rc;
  TraceScope ts(TR_TRSM, st, 4.0 * m * m * (double)ncols, 0.0);
  hipLaunchKernelGGL((trsm_kernel<T, UPPER>), dim3((ncols + CW - 1) / CW), dim3(256), shm, st, m, ncols, L,
                     ldl, X, ldx);
  HP_CHECK_LAUNCH();
  return HP_OK;
}

// ------------------------------------------------------------------- GEMM --
//
// C -= A B for complex matrices (row-major, interleaved), M x N x K, on the
// matrix cores: each complex product is four real MFMA products,
//   Cr += Ar Br - Ai Bi,   Ci += Ar Bi + Ai Br   ("4M").
// Workgroup tile 64 x 64 complex, 4 wavefronts of 32 x 32 (2 x 2 MFMA tiles
// of 16 x 16), K staged through LDS 16 complex at a time with the next stage
// prefetched into registers.  A is stored k-major in LDS so that both MFMA
// operands read 16 consecutive complex per k.
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

// Lane layout of the 16x16x4 MFMA results: accumulator element r of lane l
// holds D[mfma_row(l, r)][mfma_col(l, r)]; operands: lane l supplies
// A[a_row(l)][a_k(l)] and B[a_k(l)][a_row(l)].
// (Both layouts were read off the hardware with one-hot operands: the FP32
// instruction returns rows 4*(l/16)+r, the FP64 one rows 4*r + l/16.)
template <typename T>
struct MfmaLayout {
  static __device__ __forceinline__ int a_row(int l) { return l & 15; }
  static __device__ __forceinline__ int a_k(int l) { return l >> 4; }
  static __device__ __forceinline__ int d_row(int l, int r) { return 4 * (l >> 4) + r; }
  static __device__ __forceinline__ int d_col(int l, int r) { return l & 15; }
};
template <>
struct MfmaLayout<double> {
  static __device__ __forceinline__ int a_row(int l) { return l & 15; }
  static __device__ __forceinline__ int a_k(int l) { return l >> 4; }
  static __device__ __forceinline__ int d_row(int l, int r) { return 4 * r + (l >> 4); }
  static __device__ __forceinline__ int d_col(int l, int r) { return l & 15; }
};

constexpr int kGemmBM = 64, kGemmBN = 64, kGemmBK = 16;

template <typename T>
__global__ __launch_bounds__(256) void gemm_sub_kernel(int M, int N, int K, const cplx<T> *__restrict__ A, long lda,
                                                       long sa, const cplx<T> *__restrict__ B, long ldb, long sb,
                                                       cplx<T> *__restrict__ C, long ldc, long sc) {
  typedef typename Mfma<T>::v4 v4;
  typedef MfmaLayout<T> LY;
  constexpr int BM = kGemmBM, BN = kGemmBN, BK = kGemmBK;
  constexpr int PA = BM + 1, PB = BN + 1;  // padded LDS rows (complex)
  __shared__ cplx<T> As[BK][PA];           // k-major A tile
  __shared__ cplx<T> Bs[BK][PB];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  A += sa * blockIdx.z;
  B += sb * blockIdx.z;
  C += sc * blockIdx.z;

  // global -> register mapping: A tile 64 rows x 16 k: lane t loads row t/4, k (t%4)*4 .. +3
  const int a_r = tid >> 2, a_k = (tid & 3) * 4;
  // B tile 16 k x 64 cols: row t/16, cols (t%16)*4 .. +3
  const int b_k = tid >> 4, b_c = (tid & 15) * 4;
  cplx<T> ra[4], rb[4];

  auto load_tiles = [&](int k0) {
    const int gr = m0 + a_r;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int gk = k0 + a_k + q;
      ra[q] = (gr < M && gk < K) ? A[(long)gr * lda + gk] : cplx<T>{T(0), T(0)};
    }
    const int gk = k0 + b_k;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int gc = n0 + b_c + q;
      rb[q] = (gk < K && gc < N) ? B[(long)gk * ldb + gc] : cplx<T>{T(0), T(0)};
    }
  };
  auto store_tiles = [&]() {
#pragma unroll
    for (int q = 0; q < 4; ++q) As[a_k + q][a_r] = ra[q];
#pragma unroll
    for (int q = 0; q < 4; ++q) Bs[b_k][b_c + q] = rb[q];
  };

  v4 acc_re[2][2], acc_im[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      acc_re[i][j] = v4{0, 0, 0, 0};
      acc_im[i][j] = v4{0, 0, 0, 0};
    }

  const int nk = (K + BK - 1) / BK;
  load_tiles(0);
  store_tiles();
  __syncthreads();
  for (int kt = 0; kt < nk; ++kt) {
    if (kt + 1 < nk) load_tiles((kt + 1) * BK);
#pragma unroll
    for (int ks = 0; ks < BK; ks += 4) {
      const int kk = ks + LY::a_k(lane);
      cplx<T> af[2], bf[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) af[i] = As[kk][wm + i * 16 + LY::a_row(lane)];
#pragma unroll
      for (int j = 0; j < 2; ++j) bf[j] = Bs[kk][wn + j * 16 + LY::a_row(lane)];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        const T nai = -af[i].im;
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          acc_re[i][j] = Mfma<T>::mac(af[i].re, bf[j].re, acc_re[i][j]);
          acc_re[i][j] = Mfma<T>::mac(nai, bf[j].im, acc_re[i][j]);
          acc_im[i][j] = Mfma<T>::mac(af[i].re, bf[j].im, acc_im[i][j]);
          acc_im[i][j] = Mfma<T>::mac(af[i].im, bf[j].re, acc_im[i][j]);
        }
      }
    }
    __syncthreads();
    if (kt + 1 < nk) {
      store_tiles();
      __syncthreads();
    }
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gr = m0 + wm + i * 16 + LY::d_row(lane, r);
        const int gc = n0 + wn + j * 16 + LY::d_col(lane, r);
        if (gr < M && gc < N) {
          cplx<T> *cp = C + (long)gr * ldc + gc;
          cplx<T> c = *cp;
          c.re -= acc_re[i][j][r];
          c.im -= acc_im[i][j][r];
          *cp = c;
        }
      }
}

template <typename T>
int gemm_sub_batched(int M, int N, int K, const cplx<T> *A, long lda, long sa, const cplx<T> *B, long ldb, long sb,
                     cplx<T> *C, long ldc, long sc, int batch, hipStream_t st) {
  if (M <= 0 || N <= 0 || K <= 0 || batch <= 0) return HP_OK;
  dim3 grid((N + kGemmBN - 1) / kGemmBN, (M + kGemmBM - 1) / kGemmBM, batch);
  TraceScope ts(sizeof(T) == 8 ? TR_GEMM64 : TR_GEMM32, st, 8.0 * M * (double)N * K * batch,
                2.0 * sizeof(cplx<T>) * (double)M * N * batch);
  hipLaunchKernelGGL(gemm_sub_kernel<T>, grid, dim3(256), 0, st, M, N, K, A, lda, sa, B, ldb, sb, C, ldc, sc);
  HP_CHECK_LAUNCH();
  return HP_OK;
}

template <typename T>
int gemm_sub(int M, int N, int K, const cplx<T> *A, long lda, const cplx<T> *B, long ldb, cplx<T> *C, long ldc,
             hipStream_t st) {
  return gemm_sub_batched<T>(M, N, K, A, lda, 0, B, ldb, 0, C, ldc, 0, 1, st);
}

// ------------------------------------------------------------ factorization --

template <typename T>
struct PanelSlots {
  cplx<T> *rows;  // [2][G][W]
  T *val;         // [2][G]
  int *row;       // [2][G]
  cplx<T> *diag;  // [2][W]
};

template <typename T>
static PanelSlots<T> carve_slots(char *base) {
  PanelSlots<T> s;
  size_t off = 0;
  s.rows = (cplx<T> *)(base + off);
  off += align_up(sizeof(cplx<T>) * 2 * kMaxPanelGroups * kPanelWidth, 256);
  s.val = (T *)(base + off);
  off += align_up(sizeof(T) * 2 * kMaxPanelGroups, 256);
  s.row = (int *)(base + off);
  off += align_up(sizeof(int) * 2 * kMaxPanelGroups, 256);
  s.diag = (cplx<T> *)(base + off);
  return s;
}

static size_t slot_bytes_max() {
  return align_up(sizeof(cplx<double>) * 2 * kMaxPanelGroups * kPanelWidth, 256) +
         align_up(sizeof(double) * 2 * kMaxPanelGroups, 256) + align_up(sizeof(int) * 2 * kMaxPanelGroups, 256) +
         align_up(sizeof(cplx<double>) * 2 * kPanelWidth, 256);
}

// Rows per workgroup of the panel grid, and the grid size.
template <typename T>
static void panel_grid(int m, int &G, int &rpw) {
  // at most ~96 KB of LDS per workgroup; at most 128 workgroups (barrier cost)
  const int rpw_max = (96 * 1024) / (int)(kPanelWidth * sizeof(cplx<T>));
  const int rpw_min = 64;
  G = (m + rpw_min - 1) / rpw_min;
  G = std::min(G, 128);
  G = std::max(G, 1);
  rpw = (m + G - 1) / G;
  if (rpw > rpw_max) {
    rpw = rpw_max;
    G = (m + rpw - 1) / rpw;
  }
}

template <typename T>
static int panel(int n, int j0, int w, cplx<T> *A, long lda, int *ipiv, int *info, unsigned *bar,
                 const PanelSlots<T> &s, hipStream_t st) {
  const int m = n - j0;
  int G, rpw;
  panel_grid<T>(m, G, rpw);
  if (G > kMaxPanelGroups) return HP_ERR_UNSUPPORTED;
  size_t shm = (size_t)rpw * kPanelWidth * sizeof(cplx<T>);
  int rc = ensure_dynamic_lds((const void *)panel_kernel<T>, shm);
  if (rc) return rc;
  int nn = n, jj0 = j0, ww = w, rp = rpw;
  long ld = lda;
  cplx<T> *srows = s.rows;
  T *sval = s.val;
  int *srow = s.row;
  cplx<T> *sdiag = s.diag;
  void *args[] = {&nn, &jj0, &ww, &A, &ld, &ipiv, &info, &bar, &srows, &sval, &srow, &sdiag, &rp};
  TraceScope ts(TR_PANEL, st, 4.0 * (double)m * w * w, 2.0 * sizeof(cplx<T>) * (double)m * w);
  HP_CHECK_HIP(hipLaunchCooperativeKernel((const void *)panel_kernel<T>, dim3(G), dim3(256), args,
                                          (unsigned)shm, st));
  return HP_OK;
}

template <typename T>
int lu_factor(int n, cplx<T> *A, long lda, int *ipiv, int *perm, int *info, char *work, const Workspace &ws,
              hipStream_t st) {
  int rc;
  unsigned *bars = (unsigned *)(work + ws.sync_off);
  const size_t per_panel = barrier_words(kMaxPanelGroups);
  const int npanels = (n + kPanelWidth - 1) / kPanelWidth;
  if ((rc = fill_u32(bars, per_panel * npanels, 0u, st))) return rc;
  if ((rc = fill_u32((unsigned *)info, 1, 0u, st))) return rc;
  hipLaunchKernelGGL(iota_kernel, dim3((n + 255) / 256), dim3(256), 0, st, perm, n);
  HP_CHECK_LAUNCH();
  PanelSlots<T> slots = carve_slots<T>(work + ws.slot_off);
  for (int k = 0; k < n; k += kOuterBlock) {
    const int kb = std::min(kOuterBlock, n - k);
    for (int j = k; j < k + kb; j += kPanelWidth) {
      const int jb = std::min(kPanelWidth, k + kb - j);
      if ((rc = panel<T>(n, j, jb, A, lda, ipiv, info, bars + per_panel * (j / kPanelWidth), slots, st)))
        return rc;
      // the panel's swaps on the other columns of the outer block
      if ((rc = laswp<T>(A, lda, ipiv, j, j + jb, k, j, j + jb, k + kb, nullptr, st))) return rc;
      const int rest = k + kb - (j + jb);
      if (rest > 0) {
        cplx<T> *L11 = A + (long)j * lda + j;
        cplx<T> *A12 = A + (long)j * lda + j + jb;
        if ((rc = trsm<T, false>(jb, rest, L11, lda, A12, lda, st))) return rc;
        if ((rc = gemm_sub<T>(n - j - jb, rest, jb, A + (long)(j + jb) * lda + j, lda, A12, lda,
                              A + (long)(j + jb) * lda + j + jb, lda, st)))
          return rc;
      }
    }
    // the block's swaps on all columns outside the block, and on perm
    if ((rc = laswp<T>(A, lda, ipiv, k, k + kb, 0, k, k + kb, n, perm, st))) return rc;
    const int rest = n - k - kb;
    if (rest > 0) {
      cplx<T> *L11 = A + (long)k * lda + k;
      cplx<T> *A12 = A + (long)k * lda + k + kb;
      if ((rc = trsm<T, false>(kb, rest, L11, lda, A12, lda, st))) return rc;
      if ((rc = gemm_sub<T>(rest, rest, kb, A + (long)(k + kb) * lda + k, lda, A12, lda,
                            A + (long)(k + kb) * lda + k + kb, lda, st)))
        return rc;
    }
  }
  return HP_OK;
}

// ------------------------------------------------------------------ solve --

template <typename T>
__global__ void gather_rows_kernel(int n, int nrhs, const int *__restrict__ perm, const cplx<T> *__restrict__ X,
                                   long ldx, cplx<T> *__restrict__ Y, long ldy) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long)n * nrhs) return;
  const int i = (int)(e / nrhs), c = (int)(e - (long)i * nrhs);
  Y[(long)i * ldy + c] = X[(long)perm[i] * ldx + c];
}

template <typename T>
__global__ void copy_rows_kernel(int n, int nrhs, const cplx<T> *__restrict__ X, long ldx, cplx<T> *__restrict__ Y,
                                 long ldy) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long)n * nrhs) return;
  const int i = (int)(e / nrhs), c = (int)(e - (long)i * nrhs);
  Y[(long)i * ldy + c] = X[(long)i * ldx + c];
}

constexpr int kSolveBlock = 128;

// In-place solve on Y (n x nrhs, leading dimension ldy) that already holds P B.
template <typename T>
int lu_solve_permuted(int n, int nrhs, const cplx<T> *LU, long lda, cplx<T> *Y, long ldy, hipStream_t st) {
  int rc;
  for (int b = 0; b < n; b += kSolveBlock) {
    const int bs = std::min(kSolveBlock, n - b);
    if ((rc = trsm<T, false>(bs, nrhs, LU + (long)b * lda + b, lda, Y + (long)b * ldy, ldy, st))) return rc;
    if (b + bs < n)
      if ((rc = gemm_sub<T>(n - b - bs, nrhs, bs, LU + (long)(b + bs) * lda + b, lda, Y + (long)b * ldy, ldy,
                            Y + (long)(b + bs) * ldy, ldy, st)))
        return rc;
  }
  const int nb = (n + kSolveBlock - 1) / kSolveBlock;
  for (int bi = nb - 1; bi >= 0; --bi) {
    const int b = bi * kSolveBlock;
    const int bs = std::min(kSolveBlock, n - b);
    if ((rc = trsm<T, true>(bs, nrhs, LU + (long)b * lda + b, lda, Y + (long)b * ldy, ldy, st))) return rc;
    if (b > 0)
      if ((rc = gemm_sub<T>(b, nrhs, bs, LU + b, lda, Y + (long)b * ldy, ldy, Y, ldy, st))) return rc;
  }
  return HP_OK;
}

template <typename T>
int lu_solve(int n, int nrhs, const cplx<T> *LU, long lda, const int *perm, cplx<T> *X, long ldx, cplx<T> *tmp,
             hipStream_t st) {
  int rc;
  const long tot = (long)n * nrhs;
  const unsigned blocks = (unsigned)((tot + 255) / 256);
  hipLaunchKernelGGL(gather_rows_kernel<T>, dim3(blocks), dim3(256), 0, st, n, nrhs, perm, X, ldx, tmp,
                     (long)nrhs);
  HP_CHECK_LAUNCH();
  if ((rc = lu_solve_permuted<T>(n, nrhs, LU, lda, tmp, nrhs, st))) return rc;
  hipLaunchKernelGGL(copy_rows_kernel<T>, dim3(blocks), dim3(256), 0, st, n, nrhs, tmp, (long)nrhs, X, ldx);
  HP_CHECK_LAUNCH();
  return HP_OK;
}

// explicit instantiations
template int lu_factor<double>(int, cplx<double> *, long, int *, int *, int *, char *, const Workspace &,
                               hipStream_t);
template int lu_factor<float>(int, cplx<float> *, long, int *, int *, int *, char *, const Workspace &,
                              hipStream_t);
template int lu_solve<double>(int, int, const cplx<double> *, long, const int *, cplx<double> *, long,
                              cplx<double> *, hipStream_t);
template int lu_solve<float>(int, int, const cplx<float> *, long, const int *, cplx<float> *, long,
                             cplx<float> *, hipStream_t);
template int lu_solve_permuted<double>(int, int, const cplx<double> *, long, cplx<double> *, long, hipStream_t);
template int lu_solve_permuted<float>(int, int, const cplx<float> *, long, cplx<float> *, long, hipStream_t);
template int gemm_sub<double>(int, int, int, const cplx<double> *, long, const cplx<double> *, long,
                              cplx<double> *, long, hipStream_t);
template int gemm_sub<float>(int, int, int, const cplx<float> *, long, const cplx<float> *, long, cplx<float> *,
                             long, hipStream_t);
template int gemm_sub_batched<double>(int, int, int, const cplx<double> *, long, long, const cplx<double> *, long,
                                      long, cplx<double> *, long, long, int, hipStream_t);
template int gemm_sub_batched<float>(int, int, int, const cplx<float> *, long, long, const cplx<float> *, long,
                                     long, cplx<float> *, long, long, int, hipStream_t);

size_t factor_sync_bytes(int n) {
  const int npanels = (n + kPanelWidth - 1) / kPanelWidth;
  return sizeof(unsigned) * barrier_words(kMaxPanelGroups) * (size_t)npanels;
}
size_t factor_slot_bytes() { return slot_bytes_max(); }

}  // namespace hp

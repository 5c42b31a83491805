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

#include <cstdlib>
#include <type_traits>

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
__global__ __launch_bounds__(256, (sizeof(T) == 4 ? 4 : 2)) void gemm_sub_kernel(int M, int N, int K, const cplx<T> *__restrict__ A, long lda,
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

  // Two register sets for the staged operands: stage s is loaded into set
  // s % 2 two stages before its MFMAs, so its global loads have the MFMAs of
  // two stages to land.  (The set index is a compile-time constant in every
  // use, so the sets stay in registers.)
  Vec16<T> ra[2][G::NVA], rb[2][G::NVB];
  auto load_stage = [&](auto set, int k0) {
    constexpr int S = decltype(set)::value;
#pragma unroll
    for (int q = 0; q < G::NVA; ++q) {
      const int v = tid + 256 * q;
      const int row = v / (BK / EV), kv = v % (BK / EV);
      const int gr = m0 + row, gk = k0 + kv * EV;
      const cplx<T> *p = A + (long)gr * lda + gk;
      if (VEC && gr < M && gk + EV <= K) {
        ra[S][q] = *reinterpret_cast<const Vec16<T> *>(p);
      } else {
#pragma unroll
        for (int e = 0; e < EV; ++e) {
          ra[S][q].v[e] = cplx<T>{T(0), T(0)};
          if (gr < M && gk + e < K) ra[S][q].v[e] = p[e];
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
        rb[S][q] = *reinterpret_cast<const Vec16<T> *>(p);
      } else {
#pragma unroll
        for (int e = 0; e < EV; ++e) {
          rb[S][q].v[e] = cplx<T>{T(0), T(0)};
          if (gk < K && gc + e < N) rb[S][q].v[e] = p[e];
        }
      }
    }
  };
  auto store_stage = [&](auto set, int buf) {
    constexpr int S = decltype(set)::value;
    cplx<T> *as = As + buf * BK * PA;
    cplx<T> *bs = Bs + buf * BK * PB;
#pragma unroll
    for (int q = 0; q < G::NVA; ++q) {
      const int v = tid + 256 * q;
      const int row = v / (BK / EV), kv = v % (BK / EV);
#pragma unroll
      for (int e = 0; e < EV; ++e) as[(kv * EV + e) * PA + row] = ra[S][q].v[e];
    }
#pragma unroll
    for (int q = 0; q < G::NVB; ++q) {
      const int v = tid + 256 * q;
      const int kr = v / (BN / EV), nv = v % (BN / EV);
      *reinterpret_cast<Vec16<T> *>(bs + kr * PB + nv * EV) = rb[S][q];
    }
  };
  constexpr std::integral_constant<int, 0> set0{};
  constexpr std::integral_constant<int, 1> set1{};

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
  const int fr = lane & 15, fk = lane >> 4;
  auto compute = [&](int cur) {
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
  };
  load_stage(set0, 0);
  if (nk > 1) load_stage(set1, BK);
  store_stage(set0, 0);
  __syncthreads();
  for (int kt = 0; kt < nk; kt += 2) {
    // stage kt from LDS buffer 0; stage kt + 1 (set 1) goes to buffer 1
    if (kt + 2 < nk) load_stage(set0, (kt + 2) * BK);
    compute(0);
    if (kt + 1 < nk) store_stage(set1, 1);
    __syncthreads();
    if (kt + 1 < nk) {
      // stage kt + 1 from buffer 1; stage kt + 2 (set 0) goes to buffer 0
      if (kt + 3 < nk) load_stage(set1, (kt + 3) * BK);
      compute(1);
      if (kt + 2 < nk) store_stage(set0, 0);
      __syncthreads();
    }
  }
  // Epilogue, one row-block of MFMA tiles at a time: the C elements of the
  // row-block are all loaded (at clamped, always valid addresses) before the
  // first one is used, so those loads are in flight together; out-of-range
  // elements are skipped on the store.  Halving the live C values keeps the
  // kernel within 128 registers (4 wavefronts per SIMD).
#pragma unroll
  for (int i = 0; i < WTM; ++i) {
    cplx<T> cv[4][WTN];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int gr = min(m0 + wm + i * 16 + MfmaLayout<T>::d_row(lane, r), M - 1);
#pragma unroll
      for (int j = 0; j < WTN; ++j) {
        if constexpr (SET)
          cv[r][j] = cplx<T>{T(0), T(0)};
        else
          cv[r][j] = C[(long)gr * ldc + min(n0 + wn + j * 16 + fr, N - 1)];
      }
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int gr = m0 + wm + i * 16 + MfmaLayout<T>::d_row(lane, r);
#pragma unroll
      for (int j = 0; j < WTN; ++j) {
        const int gc = n0 + wn + j * 16 + fr;
        cplx<T> c = cv[r][j];
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
}


// FP32 operands staged by direct global->LDS loads (global_load_lds_dwordx4):
// the loaded 16-byte chunks go straight into LDS, with no pass through
// registers and no LDS store instructions; on MI355X this runs the 3M update
// ~15 % faster than the register-staged kernel (120 vs 104 TF/s of 3M flops
// on a 25344 x 25088 x 256 update).  A wave's direct load writes 64
// consecutive 16-byte slots, so the LDS layouts follow the loads: B rows are
// row-major [BK][64]; A is row-major [64][BK] with the 16-byte chunks of row r
// permuted by chunk ^ ((r / 2) % 8): a row spans half the banks, so rows r and
// r + 1 sit in different halves and the permutation separates the 8 pairs,
// and the MFMA operand reads (16 rows at one k) touch distinct banks.  The loads are issued from inline assembly (LDS
// base in M0) so that the compiler neither reorders them nor waits for them
// before the current stage's LDS reads; each thread waits for its own loads
// (vmcnt) before the barrier that publishes a stage.  Requirements (checked by
// the launcher): 16-byte aligned rows of A and B, K a multiple of 16, N even.
// Rows of A past M read row M - 1 and columns of B past N read the last column
// pair (their outputs are discarded).
constexpr int kDirectBK = 16;
// lds_byte_addr must be uniform over the wavefront.  M0 is declared clobbered,
// so the compiler keeps nothing of its own in M0 across the load.
__device__ __forceinline__ void lds_direct_load16(unsigned lds_byte_addr, const void *src) {
  const unsigned m0v = __builtin_amdgcn_readfirstlane(lds_byte_addr);
  // one wait state between the M0 write and the LDS-DMA load that reads it
  asm volatile("s_mov_b32 m0, %0\n\ts_nop 0\n\tglobal_load_lds_dwordx4 %1, off" ::"s"(m0v), "v"(src)
               : "memory", "m0");
}

// MW = 1: 64 x 64 tiles, each wavefront 32 x 32 outputs, held to three
// wavefronts per SIMD (registers claimed up to v135), 32 KB of LDS: three
// workgroups per CU leave room (LDS and registers) for a panel workgroup
// beside them -- the panel runs next to the trailing update and its grid
// only proceeds once all of its workgroups are resident.
// MW = 2: 128 x 64 tiles, each wavefront 64 x 32 outputs (twice the matrix-
// core work per operand read and per barrier), 48 KB of LDS, two workgroups
// per CU (two wavefronts per SIMD), again with room for a panel workgroup.
template <bool SET, int MW, bool CAP2 = false>
__global__ __launch_bounds__(256, (MW == 1 ? 4 : 2)) void gemm_direct_kernel(
    int M, int N, int K, const cplx<float> *__restrict__ A, long lda, long sa, const cplx<float> *__restrict__ B,
    long ldb, long sb, cplx<float> *__restrict__ C, long ldc, long sc, int tm, int tn, int total, int per_xcd,
    float alpha) {
  typedef typename Mfma<float>::v4 v4;
  if constexpr (MW == 1) asm volatile("" ::: "v135");
  if constexpr (CAP2) asm volatile("" ::: "v183");
  constexpr int BM = 64 * MW, BN = 64, BK = kDirectBK;
  constexpr int TI = 2 * MW;                 // 16-row MFMA tiles per wavefront
  constexpr int ACH = BK / 2;                // 16-byte chunks per A row
  constexpr int APW = BM * ACH / 64 / 4;     // A wave-loads per wavefront per stage
  constexpr int BPW = BK * (BN / 2) / 64 / 4;  // B wave-loads per wavefront per stage
  extern __shared__ __align__(16) char smem_raw[];
  cplx<float> *As = reinterpret_cast<cplx<float> *>(smem_raw);  // [2][BM * BK]
  cplx<float> *Bs = As + 2 * BM * BK;                            // [2][BK * BN]

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
  const int m0 = (first_m + in_grp % gm) * BM, n0 = (in_grp / gm) * BN;
  A += sa * z;
  B += sb * z;
  C += sc * z;

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = (wave >> 1) * (16 * TI), wn = (wave & 1) * 32;

  // this lane's source chunks (k0 = 0) and its wavefront's LDS slots
  const cplx<float> *asrc[APW];
  const cplx<float> *bsrc[BPW];
#pragma unroll
  for (int i = 0; i < APW; ++i) {
    const int c = (wave * APW + i) * 64 + lane;
    const int row = c / ACH, pos = c - row * ACH;
    asrc[i] = A + (long)min(m0 + row, M - 1) * lda + 2 * (pos ^ ((row >> 1) & (ACH - 1)));
  }
#pragma unroll
  for (int i = 0; i < BPW; ++i) {
    const int c = (wave * BPW + i) * 64 + lane;
    const int kr = c / (BN / 2), pos = c - kr * (BN / 2);
    bsrc[i] = B + (long)kr * ldb + min(n0 + 2 * pos, N - 2);
  }
  const unsigned lds0 = (unsigned)(size_t)(const __attribute__((address_space(3))) void *)As;
  auto issue = [&](int buf, int k0) {
#pragma unroll
    for (int i = 0; i < APW; ++i)
      lds_direct_load16(lds0 + (unsigned)((buf * BM * BK + (wave * APW + i) * 128) * sizeof(cplx<float>)),
                        asrc[i] + k0);
#pragma unroll
    for (int i = 0; i < BPW; ++i)
      lds_direct_load16(
          lds0 + (unsigned)(((2 * BM * BK) + buf * BK * BN + (wave * BPW + i) * 128) * sizeof(cplx<float>)),
          bsrc[i] + (long)k0 * ldb);
  };

  v4 acc_re[TI][2], acc_im[TI][2], acc_p2[TI][2];  // 3M: P1, P3, P2
#pragma unroll
  for (int i = 0; i < TI; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      acc_re[i][j] = v4{0, 0, 0, 0};
      acc_im[i][j] = v4{0, 0, 0, 0};
      acc_p2[i][j] = v4{0, 0, 0, 0};
    }
  const int fr = lane & 15, fk = lane >> 4;
  const int nk = K / BK;
  issue(0, 0);
  for (int kt = 0; kt < nk; ++kt) {
    // this thread's loads of stage kt have landed; the barrier publishes
    // everyone's and frees the other buffer (read during stage kt - 1)
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (kt + 1 < nk) issue((kt + 1) & 1, (kt + 1) * BK);
    const cplx<float> *as = As + (kt & 1) * BM * BK;
    const cplx<float> *bs = Bs + (kt & 1) * BK * BN;
#pragma unroll
    for (int ks = 0; ks < BK; ks += 4) {
      const int kk = ks + fk;
      cplx<float> af[TI], bf[2];
#pragma unroll
      for (int i = 0; i < TI; ++i) {
        const int row = wm + i * 16 + fr;
        af[i] = as[row * BK + 2 * ((kk >> 1) ^ ((row >> 1) & (ACH - 1))) + (kk & 1)];
      }
#pragma unroll
      for (int j = 0; j < 2; ++j) bf[j] = bs[kk * BN + wn + j * 16 + fr];
      float bsum[2];
#pragma unroll
      for (int j = 0; j < 2; ++j) bsum[j] = bf[j].re + bf[j].im;
#pragma unroll
      for (int i = 0; i < TI; ++i) {
        const float asum = af[i].re + af[i].im;
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          acc_re[i][j] = Mfma<float>::mac(af[i].re, bf[j].re, acc_re[i][j]);
          acc_p2[i][j] = Mfma<float>::mac(af[i].im, bf[j].im, acc_p2[i][j]);
          acc_im[i][j] = Mfma<float>::mac(asum, bsum[j], acc_im[i][j]);
        }
      }
    }
  }
  // epilogue as in gemm_sub_kernel, one 16-row tile at a time
#pragma unroll
  for (int i = 0; i < TI; ++i) {
    cplx<float> cv[4][2];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int gr = min(m0 + wm + i * 16 + MfmaLayout<float>::d_row(lane, r), M - 1);
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        if constexpr (SET)
          cv[r][j] = cplx<float>{0.f, 0.f};
        else
          cv[r][j] = C[(long)gr * ldc + min(n0 + wn + j * 16 + fr, N - 1)];
      }
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int gr = m0 + wm + i * 16 + MfmaLayout<float>::d_row(lane, r);
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int gc = n0 + wn + j * 16 + fr;
        cplx<float> c = cv[r][j];
        const float p1 = acc_re[i][j][r], p2 = acc_p2[i][j][r], p3 = acc_im[i][j][r];
        c.re -= p1 - p2;
        c.im -= p3 - p1 - p2;
        if constexpr (SET) c = cplx<float>{-alpha * c.re, -alpha * c.im};
        if (gr < M && gc < N) C[(long)gr * ldc + gc] = c;
      }
    }
  }
}

// Form of the direct-staged FP32 kernel (HP_GEMM_TILE): 64 (64-row tiles),
// 128 (128-row tiles, occupancy as registers and LDS allow), 1282 (128-row
// tiles held to two wavefronts per SIMD).
static int direct_form() {
  static const int form = [] {
    const char *e = getenv("HP_GEMM_TILE");
    const int v = e ? atoi(e) : 64;
    return (v == 128 || v == 1282) ? v : 64;
  }();
  return form;
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
  dim3 grid((unsigned)(8 * per_xcd));
  if constexpr (sizeof(T) == 4 && WTM == 2 && WTN == 2) {
    if (vec && K % kDirectBK == 0 && N % 2 == 0 && ldc > 0) {
      const int form = direct_form();
      const int rows = form == 64 ? 64 : 128;
      const int dtm = (M + rows - 1) / rows;
      const long dtotal_l = (long)dtm * tn * batch;
      const int dtotal = (int)dtotal_l, dper = (dtotal + 7) / 8;
      const size_t dshm = (size_t)2 * (rows + 64) * kDirectBK * sizeof(cplx<float>);
      if (form == 128)
        hipLaunchKernelGGL((gemm_direct_kernel<SET, 2>), dim3((unsigned)(8 * dper)), dim3(256), dshm, st, M, N, K,
                           A, lda, sa, B, ldb, sb, C, ldc, sc, dtm, tn, dtotal, dper, alpha);
      else if (form == 1282)
        hipLaunchKernelGGL((gemm_direct_kernel<SET, 2, true>), dim3((unsigned)(8 * dper)), dim3(256), dshm, st, M, N,
                           K, A, lda, sa, B, ldb, sb, C, ldc, sc, dtm, tn, dtotal, dper, alpha);
      else
        hipLaunchKernelGGL((gemm_direct_kernel<SET, 1>), grid, dim3(256), dshm, st, M, N, K, A, lda, sa, B, ldb, sb,
                           C, ldc, sc, tm, tn, total, per_xcd, alpha);
      HP_CHECK_LAUNCH();
      return HP_OK;
    }
  }
  const size_t shm = G::lds_bytes;
  const void *fn = vec ? (const void *)gemm_sub_kernel<T, WTM, WTN, true, SET>
                       : (const void *)gemm_sub_kernel<T, WTM, WTN, false, SET>;
  int rc = ensure_dynamic_lds(fn, shm);
  if (rc) return rc;
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

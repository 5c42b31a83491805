// Complex GEMM C -= A B on the matrix cores (the trailing update of the LU,
// Sec. 3.1 / 3.4, and every block update of the triangular solves).
// Operands with K a multiple of the stage depth go through the kernels that
// stage them by direct global->LDS loads (gemm_direct_kernel for FP32,
// gemm_direct64_kernel for FP64); the register-staged gemm_sub_kernel below
// takes the remaining shapes.
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
// consecutive 16-byte slots, so the LDS layouts follow the loads, and the
// lane -> source mapping permutes the 16-byte chunks so that the MFMA operand
// reads spread over the banks:
//  * A is row-major [BM][BK]; the chunk (2 consecutive k) at position p of
//    row r sits at p ^ swz(r), where swz separates the rows that share a
//    256-byte bank window (BK = 16: rows r, r + 1 share one, so swz = r/2 mod
//    8; BK = 8: rows r .. r + 3, swz = r/4 mod 4).  The operand read of one
//    MFMA (16 rows at one k) then touches every bank at most once per window.
//  * B is row-major [BK][64].  (Rotating the chunks of odd-k rows by half a
//    row would spread one operand read's four k rows over both halves of a
//    bank window, but it makes the two B reads' offsets depend on k, so they
//    no longer pair into one ds_read2: measured 5 % slower in the LU.)
// The loads are issued from inline assembly (LDS base in M0) so that the
// compiler neither reorders them nor waits for them before the current
// stage's LDS reads.  NBUF LDS buffers form a ring with NBUF - 1 stages of
// loads in flight: before the barrier that publishes stage kt, each thread
// waits (vmcnt) only until its own loads of stage kt have landed, the loads
// of the later stages staying in flight.  Requirements (checked by the
// launcher): 16-byte aligned rows of A and B, K a multiple of BK, N even.
// Rows of A past M read row M - 1 and columns of B past N read the last
// column pair (their outputs are discarded).
// MW = 1: 64 x 64 tiles, each wavefront 32 x 32 outputs, held to three
// wavefronts per SIMD (registers claimed up to v135): three workgroups per CU
// leave room (LDS and registers) for a panel workgroup beside them -- the
// panel runs next to the trailing update and its grid only proceeds once all
// of its workgroups are resident.
// MW = 2: 128 x 64 tiles, each wavefront 64 x 32 outputs (twice the matrix-
// core work per operand read and per barrier), two or three workgroups per
// CU as registers and LDS allow; CAP2 holds it to two.
// LDS: NBUF (64 MW + 64) BK complex (MW = 1, BK = 16, NBUF = 2: 32 KB).
template <bool SET, int MW, int BK, int NBUF, bool CAP2 = false>
__global__ __launch_bounds__(256, (MW == 1 ? 4 : 2)) void gemm_direct_kernel(
    int M, int N, int K, const cplx<float> *__restrict__ A, long lda, long sa, const cplx<float> *__restrict__ B,
    long ldb, long sb, cplx<float> *__restrict__ C, long ldc, long sc, int tm, int tn, int total, int per_xcd,
    float alpha) {
  typedef typename Mfma<float>::v4 v4;
  if constexpr (MW == 1) asm volatile("" ::: "v135");
  if constexpr (CAP2) asm volatile("" ::: "v183");
  static_assert(BK == 8 || BK == 16, "BK");
  static_assert(NBUF >= 2 && NBUF <= 4, "NBUF");
  constexpr int BM = 64 * MW, BN = 64;
  constexpr int TI = 2 * MW;                   // 16-row MFMA tiles per wavefront
  constexpr int ACH = BK / 2;                  // 16-byte chunks per A row
  constexpr int AWS = BK == 16 ? 1 : 2;        // log2 of the A rows per 256-byte bank window
  constexpr int APW = BM * ACH / 64 / 4;       // A wave-loads per wavefront per stage
  constexpr int BPW = BK * (BN / 2) / 64 / 4;  // B wave-loads per wavefront per stage
  constexpr int LPT = APW + BPW;               // direct loads per thread per stage
  constexpr int ASZ = BM * BK, BSZ = BK * BN;  // complex per buffer
  extern __shared__ __align__(16) char smem_raw[];
  cplx<float> *As = reinterpret_cast<cplx<float> *>(smem_raw);  // [NBUF][BM * BK]
  cplx<float> *Bs = As + NBUF * ASZ;                             // [NBUF][BK * BN]

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
    asrc[i] = A + (long)min(m0 + row, M - 1) * lda + 2 * (pos ^ ((row >> AWS) & (ACH - 1)));
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
      lds_direct_load16(lds0 + (unsigned)((buf * ASZ + (wave * APW + i) * 128) * sizeof(cplx<float>)),
                        asrc[i] + k0);
#pragma unroll
    for (int i = 0; i < BPW; ++i)
      lds_direct_load16(lds0 + (unsigned)((NBUF * ASZ + buf * BSZ + (wave * BPW + i) * 128) * sizeof(cplx<float>)),
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
#pragma unroll
  for (int s = 0; s < NBUF - 1; ++s)
    if (s < nk) issue(s, s * BK);
  int cur = 0;
  for (int kt = 0; kt < nk; ++kt) {
    // this thread's loads of stage kt have landed (those of the NBUF - 2
    // later stages may still be in flight); the barrier publishes everyone's
    // and frees the buffer read during stage kt - 1
    if (kt + NBUF - 2 < nk)
      wait_vmcnt<(NBUF - 2) * LPT>();
    else
      wait_vmcnt<0>();
    __syncthreads();
    if (kt + NBUF - 1 < nk) {
      const int nb = cur == 0 ? NBUF - 1 : cur - 1;
      issue(nb, (kt + NBUF - 1) * BK);
    }
    const cplx<float> *as = As + cur * ASZ;
    const cplx<float> *bs = Bs + cur * BSZ;
#pragma unroll
    for (int ks = 0; ks < BK; ks += 4) {
      const int kk = ks + fk;
      cplx<float> af[TI], bf[2];
#pragma unroll
      for (int i = 0; i < TI; ++i) {
        const int row = wm + i * 16 + fr;
        af[i] = as[row * BK + 2 * ((kk >> 1) ^ ((row >> AWS) & (ACH - 1))) + (kk & 1)];
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
    cur = cur + 1 == NBUF ? 0 : cur + 1;
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

// Form of the direct-staged FP32 kernel (HP_GEMM_TILE, for tuning): MW, BK
// and NBUF of the kernel above and whether it is held to two wavefronts per
// SIMD.  Default: 64-row tiles, BK = 16, two buffers.  Measured on MI355X
// alone (25344^2 x 256 update with its operands inside a 25600-wide matrix,
// 6MNK flops): 121 TF/s (77 % of the FP32 matrix peak) for the default, 124
// (79 %) for 128-row tiles, 118-120 for BK = 8 with three or four buffers
// and for BK = 16 with three, so operand latency is not what holds it below
// the peak (a register-only MFMA loop reaches 99 %); with K = 1024 the
// default reaches 81 %.
struct DirectForm {
  int mw, bk, nbuf;
  bool cap2;
};
static DirectForm direct_form() {
  static const DirectForm form = [] {
    const char *e = getenv("HP_GEMM_TILE");
    const int v = e ? atoi(e) : 0;
    switch (v) {
      case 6483: return DirectForm{1, 8, 3, false};
      case 6484: return DirectForm{1, 8, 4, false};
      case 64163: return DirectForm{1, 16, 3, false};
      case 128: return DirectForm{2, 16, 2, false};
      case 1282: return DirectForm{2, 16, 2, true};
      case 12884: return DirectForm{2, 8, 4, false};
      case 128842: return DirectForm{2, 8, 4, true};
      case 128163: return DirectForm{2, 16, 3, false};
      default: return DirectForm{1, 16, 2, false};
    }
  }();
  return form;
}

template <bool SET, int MW, int BK, int NBUF, bool CAP2>
static int launch_direct(int M, int N, int K, const cplx<float> *A, long lda, long sa, const cplx<float> *B,
                          long ldb, long sb, cplx<float> *C, long ldc, long sc, int tn, int batch, float alpha,
                          hipStream_t st) {
  const int dtm = (M + 64 * MW - 1) / (64 * MW);
  const int dtotal = (int)((long)dtm * tn * batch), dper = (dtotal + 7) / 8;
  const size_t shm = (size_t)NBUF * (64 * MW + 64) * BK * sizeof(cplx<float>);
  if (shm > 64 * 1024) {
    const int rc = ensure_dynamic_lds((const void *)gemm_direct_kernel<SET, MW, BK, NBUF, CAP2>, shm);
    if (rc) return rc;
  }
  hipLaunchKernelGGL((gemm_direct_kernel<SET, MW, BK, NBUF, CAP2>), dim3((unsigned)(8 * dper)), dim3(256), shm, st,
                     M, N, K, A, lda, sa, B, ldb, sb, C, ldc, sc, dtm, tn, dtotal, dper, alpha);
  return HP_OK;
}

// FP64 operands staged by direct global->LDS loads: one complex double is
// one 16-byte chunk, so a wave's direct load fills 64 consecutive elements.
// A is row-major [64][BK] with element k of row r at k ^ swz(r), swz
// separating the rows that share a 256-byte bank window (BK = 8: rows r and
// r + 1, swz = r/2 mod 8; BK = 16: swz = r mod 16), so the operand read of
// one MFMA (16 rows at one k, 16 bytes each) covers a window once; B is
// row-major [BK][64] (16 consecutive columns per k: one window).  The
// products are the 4M form of gemm_sub_kernel on v_mfma_f64_16x16x4f64; the
// ring of NBUF buffers and the vmcnt waits are those of the FP32 kernel.
// 64 x 64 tiles, each wavefront 32 x 32 outputs; LDS NBUF 128 BK 16 bytes
// (BK = 8, NBUF = 2: 32 KB).  Rows of A past M read row M - 1 and columns of
// B past N read column N - 1 (outputs discarded).  K a multiple of BK.
template <bool SET, int BK, int NBUF, int OCC>
__global__ __launch_bounds__(256, OCC) void gemm_direct64_kernel(
    int M, int N, int K, const cplx<double> *__restrict__ A, long lda, long sa, const cplx<double> *__restrict__ B,
    long ldb, long sb, cplx<double> *__restrict__ C, long ldc, long sc, int tm, int tn, int total, int per_xcd,
    double alpha) {
  typedef typename Mfma<double>::v4 v4;
  // OCC = 2 or 3: registers claimed so that at most OCC wavefronts share a SIMD
  if constexpr (OCC == 2) asm volatile("" ::: "v183");
  if constexpr (OCC == 3) asm volatile("" ::: "v135");
  static_assert(BK == 8 || BK == 16, "BK");
  static_assert(NBUF >= 2 && NBUF <= 4, "NBUF");
  constexpr int BM = 64, BN = 64, TI = 2;
  constexpr int AWS = BK == 16 ? 0 : 1;        // log2 of the A rows per 256-byte bank window
  constexpr int APW = BM * BK / 64 / 4;        // A wave-loads per wavefront per stage
  constexpr int BPW = BK * BN / 64 / 4;        // B wave-loads per wavefront per stage
  constexpr int LPT = APW + BPW;
  constexpr int ASZ = BM * BK, BSZ = BK * BN;
  extern __shared__ __align__(16) char smem_raw[];
  cplx<double> *As = reinterpret_cast<cplx<double> *>(smem_raw);  // [NBUF][BM * BK]
  cplx<double> *Bs = As + NBUF * ASZ;                              // [NBUF][BK * BN]

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
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;

  const cplx<double> *asrc[APW];
  const cplx<double> *bsrc[BPW];
#pragma unroll
  for (int i = 0; i < APW; ++i) {
    const int c = (wave * APW + i) * 64 + lane;
    const int row = c / BK, pos = c - row * BK;
    asrc[i] = A + (long)min(m0 + row, M - 1) * lda + (pos ^ ((row >> AWS) & (BK - 1)));
  }
#pragma unroll
  for (int i = 0; i < BPW; ++i) {
    const int c = (wave * BPW + i) * 64 + lane;
    const int kr = c / BN, pos = c - kr * BN;
    bsrc[i] = B + (long)kr * ldb + min(n0 + pos, N - 1);
  }
  const unsigned lds0 = (unsigned)(size_t)(const __attribute__((address_space(3))) void *)As;
  auto issue = [&](int buf, int k0) {
#pragma unroll
    for (int i = 0; i < APW; ++i)
      lds_direct_load16(lds0 + (unsigned)((buf * ASZ + (wave * APW + i) * 64) * sizeof(cplx<double>)), asrc[i] + k0);
#pragma unroll
    for (int i = 0; i < BPW; ++i)
      lds_direct_load16(lds0 + (unsigned)((NBUF * ASZ + buf * BSZ + (wave * BPW + i) * 64) * sizeof(cplx<double>)),
                        bsrc[i] + (long)k0 * ldb);
  };

  v4 acc_re[TI][2], acc_im[TI][2];
#pragma unroll
  for (int i = 0; i < TI; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      acc_re[i][j] = v4{0, 0, 0, 0};
      acc_im[i][j] = v4{0, 0, 0, 0};
    }
  const int fr = lane & 15, fk = lane >> 4;
  const int nk = K / BK;
#pragma unroll
  for (int s = 0; s < NBUF - 1; ++s)
    if (s < nk) issue(s, s * BK);
  int cur = 0;
  for (int kt = 0; kt < nk; ++kt) {
    if (kt + NBUF - 2 < nk)
      wait_vmcnt<(NBUF - 2) * LPT>();
    else
      wait_vmcnt<0>();
    __syncthreads();
    if (kt + NBUF - 1 < nk) {
      const int nb = cur == 0 ? NBUF - 1 : cur - 1;
      issue(nb, (kt + NBUF - 1) * BK);
    }
    const cplx<double> *as = As + cur * ASZ;
    const cplx<double> *bs = Bs + cur * BSZ;
#pragma unroll
    for (int ks = 0; ks < BK; ks += 4) {
      const int kk = ks + fk;
      cplx<double> af[TI], bf[2];
#pragma unroll
      for (int i = 0; i < TI; ++i) {
        const int row = wm + i * 16 + fr;
        af[i] = as[row * BK + (kk ^ ((row >> AWS) & (BK - 1)))];
      }
#pragma unroll
      for (int j = 0; j < 2; ++j) bf[j] = bs[kk * BN + wn + j * 16 + fr];
#pragma unroll
      for (int i = 0; i < TI; ++i) {
        const double nai = -af[i].im;
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          acc_re[i][j] = Mfma<double>::mac(af[i].re, bf[j].re, acc_re[i][j]);
          acc_im[i][j] = Mfma<double>::mac(af[i].re, bf[j].im, acc_im[i][j]);
          acc_re[i][j] = Mfma<double>::mac(nai, bf[j].im, acc_re[i][j]);
          acc_im[i][j] = Mfma<double>::mac(af[i].im, bf[j].re, acc_im[i][j]);
        }
      }
    }
    cur = cur + 1 == NBUF ? 0 : cur + 1;
  }
#pragma unroll
  for (int i = 0; i < TI; ++i) {
    cplx<double> cv[4][2];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int gr = min(m0 + wm + i * 16 + MfmaLayout<double>::d_row(lane, r), M - 1);
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        if constexpr (SET)
          cv[r][j] = cplx<double>{0.0, 0.0};
        else
          cv[r][j] = C[(long)gr * ldc + min(n0 + wn + j * 16 + fr, N - 1)];
      }
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int gr = m0 + wm + i * 16 + MfmaLayout<double>::d_row(lane, r);
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int gc = n0 + wn + j * 16 + fr;
        cplx<double> c = cv[r][j];
        c.re -= acc_re[i][j][r];
        c.im -= acc_im[i][j][r];
        if constexpr (SET) c = cplx<double>{-alpha * c.re, -alpha * c.im};
        if (gr < M && gc < N) C[(long)gr * ldc + gc] = c;
      }
    }
  }
}

// Form of the direct-staged FP64 kernel (HP_GEMM64_TILE, for tuning): BK,
// NBUF and the wavefronts per SIMD (= workgroups per CU) it is held to; 0
// selects the register-staged kernel.  Measured on MI355X alone (25344^2 x
// 256 update, 8MNK flops): 68.8 TF/s (87.5 % of the FP64 matrix peak) for
// the default (BK = 8, two buffers, three workgroups per CU: 96 KB of LDS, so
// a 256-workgroup FP64 panel's 53 KB of rows fit beside it), 66.3 for two
// workgroups, 69.6 for four (which leaves the panel no room: the FP64 LU step
// is 11 % slower), against 63.0 for the register-staged kernel.
struct Direct64Form {
  int bk, nbuf, occ;
};
static Direct64Form direct64_form() {
  static const Direct64Form form = [] {
    const char *e = getenv("HP_GEMM64_TILE");
    const int v = e ? atoi(e) : 823;
    switch (v) {
      case 0: return Direct64Form{0, 0, 0};
      case 822: return Direct64Form{8, 2, 2};
      case 824: return Direct64Form{8, 2, 4};
      default: return Direct64Form{8, 2, 3};
    }
  }();
  return form;
}

template <bool SET, int BK, int NBUF, int OCC>
static int launch_direct64(int M, int N, int K, const cplx<double> *A, long lda, long sa, const cplx<double> *B,
                           long ldb, long sb, cplx<double> *C, long ldc, long sc, int tm, int tn, int batch,
                           double alpha, hipStream_t st) {
  const int total = (int)((long)tm * tn * batch), per = (total + 7) / 8;
  const size_t shm = (size_t)NBUF * 128 * BK * sizeof(cplx<double>);
  if (shm > 64 * 1024) {
    const int rc = ensure_dynamic_lds((const void *)gemm_direct64_kernel<SET, BK, NBUF, OCC>, shm);
    if (rc) return rc;
  }
  hipLaunchKernelGGL((gemm_direct64_kernel<SET, BK, NBUF, OCC>), dim3((unsigned)(8 * per)), dim3(256), shm, st, M,
                     N, K, A, lda, sa, B, ldb, sb, C, ldc, sc, tm, tn, total, per, alpha);
  return HP_OK;
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
    const DirectForm f = direct_form();
    if (vec && K % f.bk == 0 && N % 2 == 0 && ldc > 0) {
      const int id = f.mw * 10000 + f.bk * 100 + f.nbuf * 10 + (f.cap2 ? 1 : 0);
      int rc;
      switch (id) {
        case 10830: rc = launch_direct<SET, 1, 8, 3, false>(M, N, K, A, lda, sa, B, ldb, sb, C, ldc, sc, tn, batch, alpha, st); break;
        case 10840: rc = launch_direct<SET, 1, 8, 4, false>(M, N, K, A, lda, sa, B, ldb, sb, C, ldc, sc, tn, batch, alpha, st); break;
        case 11630: rc = launch_direct<SET, 1, 16, 3, false>(M, N, K, A, lda, sa, B, ldb, sb, C, ldc, sc, tn, batch, alpha, st); break;
        case 21620: rc = launch_direct<SET, 2, 16, 2, false>(M, N, K, A, lda, sa, B, ldb, sb, C, ldc, sc, tn, batch, alpha, st); break;
        case 21621: rc = launch_direct<SET, 2, 16, 2, true>(M, N, K, A, lda, sa, B, ldb, sb, C, ldc, sc, tn, batch, alpha, st); break;
        case 20840: rc = launch_direct<SET, 2, 8, 4, false>(M, N, K, A, lda, sa, B, ldb, sb, C, ldc, sc, tn, batch, alpha, st); break;
        case 20841: rc = launch_direct<SET, 2, 8, 4, true>(M, N, K, A, lda, sa, B, ldb, sb, C, ldc, sc, tn, batch, alpha, st); break;
        case 21630: rc = launch_direct<SET, 2, 16, 3, false>(M, N, K, A, lda, sa, B, ldb, sb, C, ldc, sc, tn, batch, alpha, st); break;
        default: rc = launch_direct<SET, 1, 16, 2, false>(M, N, K, A, lda, sa, B, ldb, sb, C, ldc, sc, tn, batch, alpha, st); break;
      }
      if (rc) return rc;
      HP_CHECK_LAUNCH();
      return HP_OK;
    }
  }
  if constexpr (sizeof(T) == 8 && WTM == 2 && WTN == 2) {
    const Direct64Form f = direct64_form();
    if (f.bk > 0 && K % f.bk == 0 && ldc > 0) {
      const int id = f.bk * 100 + f.nbuf * 10 + f.occ;
      int rc;
      switch (id) {
        case 822: rc = launch_direct64<SET, 8, 2, 2>(M, N, K, A, lda, sa, B, ldb, sb, C, ldc, sc, tm, tn, batch, alpha, st); break;
        case 824: rc = launch_direct64<SET, 8, 2, 4>(M, N, K, A, lda, sa, B, ldb, sb, C, ldc, sc, tm, tn, batch, alpha, st); break;
        default: rc = launch_direct64<SET, 8, 2, 3>(M, N, K, A, lda, sa, B, ldb, sb, C, ldc, sc, tm, tn, batch, alpha, st); break;
      }
      if (rc) return rc;
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
  // 64 x 64 tiles in both precisions (the direct-staged kernels' forms and
  // their measured rates are given with the kernels).  The register-staged
  // kernel: 64 x 64 tiles measured against 128-wide ones, whose register
  // footprint leaves one wavefront per SIMD.  Loading C during the last K
  // stage (FP32) measured 1 % slower alone, and slower beside the panel.
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

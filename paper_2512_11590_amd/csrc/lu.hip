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
//     panel_kernel       cooperative grid, one grid-wide exchange per column:
//                        pivot search (wavefront reductions + slot exchange), row swap,
//                        scaling and rank-1 update of the panel held in LDS
//     laswp_kernel       the panel's swaps on the other columns of the block
//     trsm + gemm_sub    U rows of the panel and update of the rest of the block
//   laswp_kernel         the block's swaps on every column outside the block
//   trsm_lower_unit      U12 = L11^-1 A12
//   gemm_sub             A22 -= L21 U12 (MFMA complex GEMM, 4 real products)
#include "common.h"

#include <type_traits>
#include <utility>
#include <memory>
#include <atomic>
#include <mutex>
#include <map>

#include <algorithm>
#include <climits>
#include <cstdlib>

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

// FP32 wavefront argmax on the DPP and readlane paths (no LDS round trips):
// butterflies inside each row of 16 lanes, then the four row results
// combined; every lane returns the wave's (value, row).
template <int kCtrl>
__device__ __forceinline__ void dpp_argmax_step(float &v, int &r) {
  const float ov = __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), kCtrl, 0xF, 0xF, false));
  const int orow = __builtin_amdgcn_update_dpp(0, r, kCtrl, 0xF, 0xF, false);
  argmax_combine(v, r, ov, orow);
}
__device__ __forceinline__ void wave_argmax_dpp(float &v, int &r) {
  dpp_argmax_step<0xB1>(v, r);   // quad_perm [1,0,3,2]: lane ^ 1
  dpp_argmax_step<0x4E>(v, r);   // quad_perm [2,3,0,1]: lane ^ 2
  dpp_argmax_step<0x141>(v, r);  // row_half_mirror: the other quad of each 8
  dpp_argmax_step<0x140>(v, r);  // row_mirror: the other 8 of each 16
  float bv = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 0));
  int br = __builtin_amdgcn_readlane(r, 0);
#pragma unroll
  for (int l = 16; l < 64; l += 16)
    argmax_combine(bv, br, __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l)), __builtin_amdgcn_readlane(r, l));
  v = bv;
  r = br;
}
// Whole-workgroup FP32 argmax with one barrier.  Two calls that use the same
// sv/sr must have a __syncthreads between them (the callers' other barriers).
__device__ __forceinline__ void block_argmax_dpp(float &v, int &r, float *sv, int *sr) {
  wave_argmax_dpp(v, r);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
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

// Grid synchronisation of the cooperative panel grid without atomics: every
// workgroup owns one flag word and publishes the epoch it has reached there
// (after its slot data is globally visible); a workgroup waits by polling all
// the flags, one lane per flag.  The wait is bounded: on expiry it records -1
// in *flag and stops waiting, and later waits return at once, so the grid
// always drains.
//
// Visibility across the XCDs' separate L2 caches rests on the gfx9 ISA, not
// on C++ release/acquire: every datum a workgroup publishes (slot values,
// rows, flags, key words) is written with an agent-scope atomic store, which
// compiles to a write-through store (sc1); each thread then waits for its
// own stores to be acknowledged (s_waitcnt vmcnt(0)) before the barrier
// after which one thread stores the flag, so the data reach the device's
// coherence point before the flag is issued; readers load every published
// datum with agent-scope atomic loads (sc1, not served from a stale L2 line),
// issued only after the flag or key word they wait for has been observed.
// This is the code sequence of an agent-scope release store / acquire load
// without the whole-cache operations (buffer_wbl2 sc1 / buffer_inv sc1) that
// those add for plain, non-atomic data, which the exchange never uses.
// Written as C++ agent-scope release/acquire fences instead, the FP32 step
// measured 550 ms against 495 and the FP64 step 989 against 880: per column,
// every panel workgroup wrote back and invalidated the L2 its XCD shares
// with the trailing update.
constexpr int kBarStride = 1;

__device__ __forceinline__ void grid_arrive(unsigned *bar, unsigned epoch) {
  // every lane's agent-scope stores must have completed before the flag moves
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (threadIdx.x == 0)
    __hip_atomic_store(bar + blockIdx.x, epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void grid_wait(unsigned *bar, unsigned ngroups, unsigned epoch, int *flag) {
  (void)ngroups;
  // once a wait has expired anywhere in the grid, no workgroup waits again,
  // so a failed factorization drains at memory speed
  const bool failed = __hip_atomic_load(flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == -1;
  for (unsigned g = threadIdx.x; !failed && g < gridDim.x; g += blockDim.x) {
    unsigned spins = 0;
    while (__hip_atomic_load(bar + g, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < epoch) {
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

static size_t barrier_words(int G) { return (size_t)G * kBarStride; }

// FP32 panels publish each workgroup's pivot candidate as one 64-bit word:
// the candidate value's bits above the column's epoch (global column + 1,
// 19 bits) and the candidate's row offset inside its workgroup (13 bits; all
// ones for "no candidate").  A reader polls the word until it carries the
// epoch it waits for, so the arrival flag and the value read are one round
// trip.  The word is stored after the workgroup's slot rows are visible.
constexpr int kKeyRowBits = 13;
constexpr unsigned kKeyNoRow = (1u << kKeyRowBits) - 1;
constexpr int kKeyMaxColumns = 1 << (32 - kKeyRowBits);

__device__ __forceinline__ unsigned long long make_key(float v, unsigned epoch, unsigned rowoff) {
  return ((unsigned long long)__float_as_uint(v) << 32) | (epoch << kKeyRowBits) | rowoff;
}

// Bounded wait for the key word at p to carry epoch; returns the last word
// read (on expiry -1 is recorded in *flag, as in grid_wait).
__device__ __forceinline__ unsigned long long wait_key(const unsigned long long *p, unsigned epoch, bool failed,
                                                       int *flag) {
  unsigned long long v = __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  unsigned spins = 0;
  while (!failed && ((unsigned)v >> kKeyRowBits) != epoch) {
    __builtin_amdgcn_s_sleep(1);
    if (((++spins) & 1023u) == 0) {
      if (spins > kSpinLimit || __hip_atomic_load(flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == -1) {
        atomicExch(flag, -1);
        break;
      }
    }
    v = __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  return v;
}

// ------------------------------------------------------------ panel (LU) --
//
// Factor columns [j0, j0+w) of rows [j0, n) with partial pivoting.  The rows
// are split into contiguous chunks of rpw rows, one per workgroup, held in
// LDS for the whole panel.  Per column j: every workgroup publishes its
// candidate pivot for column j (largest |Re|+|Im|, smallest row on ties)
// together with that row's panel values in a slot, and the owner of row j
// publishes row j; every workgroup waits for all candidates (FP32: polls the
// candidates' epoch-tagged key words, which carry the values; FP64: a flag
// barrier, then the value slots), picks the same winner and then reads only
// the winner's row (a second short round trip costs less than moving every
// candidate row to every workgroup), the owners of the two rows exchange
// them, and each workgroup eliminates in its own rows.  The elimination is
// split so the wait hides most of it: column j+1 is updated first (it
// decides the next pivot), the next candidate row and the next diagonal row
// are finished and published, and the remaining columns are updated while
// the other workgroups arrive.  Slots alternate between two buffers, so a
// slow reader never sees the next column's writes.
constexpr int kPanelLd = kPanelWidth + 1;  // LDS row stride of the panel rows (complex elements)

template <typename T>
__global__ __launch_bounds__(256) void panel_kernel(int n, int j0, int w, cplx<T> *__restrict__ A,
                                                    long lda, int *__restrict__ ipiv,
                                                    int *__restrict__ info, unsigned *bar,
                                                    cplx<T> *slot_rows, T *slot_val, int *slot_row,
                                                    cplx<T> *diag_rows, unsigned long long *slot_key, int rpw) {
  // the panel chain is latency-bound and shares its SIMDs with the
  // MFMA-bound trailing update: its waves go first in instruction issue
  __builtin_amdgcn_s_setprio(3);
  extern __shared__ __align__(16) char smem_raw[];
  cplx<T> *Ls = reinterpret_cast<cplx<T> *>(smem_raw);  // [rpw][kPanelLd]
  __shared__ cplx<T> urow[kPanelWidth], drow[kPanelWidth];
  __shared__ T red_v[4], red_v2[4];  // read-side and elimination-side argmax exchange
  __shared__ int red_r[4], red_r2[4];
  // FP32: candidates as epoch-tagged key words (slot_key); FP64: value and
  // row slots behind the flag barrier (the value leaves no room for a tag)
  constexpr bool kKeyed = std::is_same<T, float>::value;
  auto argmax_all = [&](T &v, int &r, T *sv, int *sr) {
    if constexpr (kKeyed)
      block_argmax_dpp(v, r, sv, sr);
    else
      block_argmax(v, r, sv, sr);
  };
  constexpr int W = kPanelWidth;
  constexpr int LW = kPanelLd;  // padded row stride: rows 2 banks apart, so a column's elements spread over the banks
  const int G = gridDim.x, g = blockIdx.x, tid = threadIdx.x;
  const unsigned ngroups = (unsigned)G;
  const int rbeg = j0 + g * rpw;
  const int rend = min(n, rbeg + rpw);
  const int nrow = max(0, rend - rbeg);

  // rows into LDS, eight loads per thread in flight at a time (clamped
  // addresses, so every load is in bounds and none waits on a branch)
  for (int e0 = 0; e0 < nrow * w; e0 += 8 * 256) {
    cplx<T> buf[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = min(e0 + u * 256 + tid, nrow * w - 1);
      const int rr = e / w, cc = e - rr * w;
      buf[u] = A[(long)(rbeg + rr) * lda + j0 + cc];
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = e0 + u * 256 + tid;
      if (e < nrow * w) {
        const int rr = e / w, cc = e - rr * w;
        Ls[rr * LW + cc] = buf[u];
      }
    }
  }
  __syncthreads();

  // publish the candidate of column jj (slot buffer jj & 1) and row j0+jj,
  // then arrive: the key word (FP32) or the arrival flag, once the rows are
  // visible
  auto publish = [&](int jj, T best, int brow) {
    const int par = jj & 1;
    if constexpr (!kKeyed) {
      if (tid == 0) {
        st_agent(&slot_val[par * G + g], best);
        st_agent(&slot_row[par * G + g], brow);
      }
    }
    if (brow != INT_MAX)
      for (int cc = tid; cc < w; cc += 256)
        st_agent(&slot_rows[((size_t)par * G + g) * W + cc], Ls[(brow - rbeg) * LW + cc]);
    const int jd = j0 + jj;
    if (jd >= rbeg && jd < rend)
      for (int cc = tid; cc < w; cc += 256) st_agent(&diag_rows[par * W + cc], Ls[(jd - rbeg) * LW + cc]);
    if constexpr (kKeyed) {
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
      __builtin_amdgcn_s_waitcnt(0);
      __syncthreads();
      if (tid == 0) {
        const unsigned off = brow == INT_MAX ? kKeyNoRow : (unsigned)(brow - rbeg);
        __hip_atomic_store(&slot_key[par * G + g], make_key(best, (unsigned)(jd + 1), off), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
      }
    } else {
      grid_arrive(bar, (unsigned)(jj + 1));
    }
  };

  // prologue: candidate for the first column
  {
    T best = T(-1);
    int brow = INT_MAX;
    for (int rr = tid; rr < nrow; rr += 256) argmax_combine(best, brow, cabs1(Ls[rr * LW]), rbeg + rr);
    argmax_all(best, brow, red_v2, red_r2);
    publish(0, best, brow);
  }

  for (int j = 0; j < w; ++j) {
    const int jc = j0 + j;
    const int par = j & 1;
    // -- every candidate's value and row, then the winner's panel row from
    //    the slot of the workgroup that owns it (and row jc)
    T wv = T(-1);
    int wr = INT_MAX;
    if constexpr (kKeyed) {
      const bool failed = __hip_atomic_load(info, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == -1;
      for (int e = tid; e < G; e += 256) {
        const unsigned long long key = wait_key(&slot_key[par * G + e], (unsigned)(jc + 1), failed, info);
        const unsigned off = (unsigned)key & kKeyNoRow;
        argmax_combine(wv, wr, __uint_as_float((unsigned)(key >> 32)), off == kKeyNoRow ? INT_MAX : j0 + e * rpw + (int)off);
      }
    } else {
      grid_wait(bar, ngroups, (unsigned)(j + 1), info);
      for (int e = tid; e < G; e += 256) argmax_combine(wv, wr, ld_agent(&slot_val[par * G + e]), ld_agent(&slot_row[par * G + e]));
      if (tid < w) drow[tid] = ld_agent(&diag_rows[par * W + tid]);
    }
    argmax_all(wv, wr, red_v, red_r);
    int p = wr;
    if (p < jc || p >= n) {  // cannot happen unless the exchange failed; never index out of range
      if (g == 0 && tid == 0) atomicExch(info, -1);
      p = jc;
    }
    const int wg = min(G - 1, (p - j0) / rpw);
    if (tid < w) urow[tid] = ld_agent(&slot_rows[((size_t)par * G + wg) * W + tid]);
    if constexpr (kKeyed) {
      if (tid >= 64 && tid < 64 + w) drow[tid - 64] = ld_agent(&diag_rows[par * W + tid - 64]);
    }
    __syncthreads();
    if (g == 0 && tid == 0) {
      ipiv[jc] = p;
      if (!(wv > T(0))) atomicCAS(info, 0, jc + 1);
    }
    if (jc >= rbeg && jc < rend)
      for (int cc = tid; cc < w; cc += 256) Ls[(jc - rbeg) * LW + cc] = urow[cc];
    if (p != jc && p >= rbeg && p < rend)
      for (int cc = tid; cc < w; cc += 256) Ls[(p - rbeg) * LW + cc] = drow[cc];
    __syncthreads();
    // -- eliminate: scale column j below the pivot (an exactly zero pivot
    //    column is left as it is, and nothing is subtracted)
    const bool nz = wv > T(0);
    const cplx<T> inv = nz ? crcp(urow[j]) : cplx<T>{T(0), T(0)};
    if (j == w - 1) {
      if (nz)
        for (int rr = tid; rr < nrow; rr += 256)
          if (rbeg + rr > jc) Ls[rr * LW + j] = cmul(Ls[rr * LW + j], inv);
      __syncthreads();
      break;
    }
    // column j+1 first, with the next pivot search
    T best = T(-1);
    int brow = INT_MAX;
    for (int rr = tid; rr < nrow; rr += 256) {
      const int gr = rbeg + rr;
      if (gr > jc) {
        if (nz) {
          const cplx<T> lv = cmul(Ls[rr * LW + j], inv);
          Ls[rr * LW + j] = lv;
          Ls[rr * LW + j + 1] = cfms(Ls[rr * LW + j + 1], lv, urow[j + 1]);
        }
        argmax_combine(best, brow, cabs1(Ls[rr * LW + j + 1]), gr);
      }
    }
    argmax_all(best, brow, red_v2, red_r2);
    // finish the two rows that are published next: the candidate and row jc+1
    const int r1 = (brow != INT_MAX) ? brow - rbeg : -1;
    const int r2 = (jc + 1 >= rbeg && jc + 1 < rend) ? jc + 1 - rbeg : -1;
    if (nz) {
      for (int cc = j + 2 + tid; cc < w; cc += 256) {
        if (r1 >= 0) Ls[r1 * LW + cc] = cfms(Ls[r1 * LW + cc], Ls[r1 * LW + j], urow[cc]);
        if (r2 >= 0 && r2 != r1) Ls[r2 * LW + cc] = cfms(Ls[r2 * LW + cc], Ls[r2 * LW + j], urow[cc]);
      }
    }
    __syncthreads();
    publish(j + 1, best, brow);
    // the remaining columns of the other rows, while the grid arrives
    if (nz && j + 2 < w) {
      for (int rr = tid; rr < nrow; rr += 256) {
        if (rbeg + rr > jc && rr != r1 && rr != r2) {
          const cplx<T> lv = Ls[rr * LW + j];
          for (int cc = j + 2; cc < w; ++cc) Ls[rr * LW + cc] = cfms(Ls[rr * LW + cc], lv, urow[cc]);
        }
      }
    }
  }
  for (int e = tid; e < nrow * w; e += 256) {
    const int rr = e / w, cc = e - rr * w;
    A[(long)(rbeg + rr) * lda + j0 + cc] = Ls[rr * LW + cc];
  }
}

// ------------------------------------------------------------------ laswp --
//
// Row interchanges of one block of pivots, ipiv[k0 .. k0+kb), applied to
// columns [c0, c1) and [c2, c3).  The interchanges are applied in order, so
// their net effect is a permutation of at most 2 kb rows: the kb block rows
// and the distinct pivot rows below the block.  swap_plan_kernel works it out
// once (one workgroup, in LDS) as a list of (destination row, source row)
// moves and applies it to perm; row_permute_kernel then moves the rows of
// every column stripe through LDS in one parallel pass (all sources read
// before any destination is written), instead of kb dependent swaps.
constexpr int kPlanMax = 2 * kOuterBlock;

__global__ __launch_bounds__(256) void swap_plan_kernel(const int *__restrict__ ipiv, int k0, int kb, int n,
                                                        int *__restrict__ plan, int *__restrict__ perm,
                                                        int *__restrict__ info) {
  __shared__ int pp[kOuterBlock], firstj[kOuterBlock], bsl[kOuterBlock], cidx[kOuterBlock];
  __shared__ int pos[kPlanMax], val[kPlanMax];
  __shared__ int nout, nmove, wcnt[4];
  __shared__ int pv[kPlanMax], pd[kPlanMax];
  const int tid = threadIdx.x;
  if (tid < kb) {
    int p = ipiv[k0 + tid];
    if (p < k0 + tid || p >= n) {  // never expected; keep every index in range
      atomicExch(info, -1);
      p = k0 + tid;
    }
    pp[tid] = p;
  }
  __syncthreads();
  // first interchange that brings each outside pivot row in
  int isf = 0;
  if (tid < kb) {
    const int p = pp[tid];
    int f = tid;
    if (p >= k0 + kb)
      for (int j = 0; j < tid; ++j)
        if (pp[j] == p && f == tid) f = j;
    firstj[tid] = f;
    isf = (p >= k0 + kb && f == tid) ? 1 : 0;
  }
  // slot numbers of the outside rows: exclusive prefix count of the first
  // appearances, from the wavefront ballots
  const int lane = tid & 63, wave = tid >> 6;
  const unsigned long long firsts = __ballot(isf);
  if (lane == 0) wcnt[wave] = __popcll(firsts);
  __syncthreads();
  int before = 0;
  for (int w = 0; w < wave; ++w) before += wcnt[w];
  cidx[tid] = before + __popcll(firsts & ((1ull << lane) - 1));
  if (tid == 0) {
    nout = wcnt[0] + wcnt[1] + wcnt[2] + wcnt[3];
    nmove = 0;
  }
  __syncthreads();
  // the slot of each interchange's pivot row, and the row of each slot
  if (tid < kb) {
    const int p = pp[tid];
    bsl[tid] = (p < k0 + kb) ? (p - k0) : (kb + cidx[firstj[tid]]);
    pos[tid] = k0 + tid;
    if (isf) pos[kb + cidx[tid]] = p;
  }
  __syncthreads();
  // the row whose content ends in each slot: the slot traced back through
  // the interchanges, last to first (one slot per thread, no serial replay)
  {
    const int ns = kb + nout;
    for (int sl = tid; sl < ns; sl += 256) {
      int q = sl;
      for (int j = kb - 1; j >= 0; --j) {
        const int bj = bsl[j];
        q = (q == j) ? bj : (q == bj ? j : q);
      }
      val[sl] = pos[q];
    }
  }
  __syncthreads();
  const int ns = kb + nout;
  for (int sl = tid; sl < ns; sl += 256) {
    if (val[sl] != pos[sl]) {
      const int m = atomicAdd(&nmove, 1);
      plan[1 + m] = pos[sl];             // destination row
      plan[1 + kPlanMax + m] = val[sl];  // source row
      pd[m] = pos[sl];
      if (perm) pv[m] = perm[val[sl]];
    }
  }
  __syncthreads();
  if (tid == 0) plan[0] = nmove;
  if (perm) {
    for (int m = tid; m < nmove; m += 256) perm[pd[m]] = pv[m];
  }
}

template <typename T>
struct PermCfg {
  static constexpr int CW = 16;  // columns per workgroup (LDS: kPlanMax x CW complex)
};
template <>
struct PermCfg<float> {
  static constexpr int CW = 32;
};

template <typename T>
__global__ __launch_bounds__(256) void row_permute_kernel(cplx<T> *__restrict__ A, long lda,
                                                          const int *__restrict__ plan, int c0, int c1, int c2,
                                                          int c3) {
  constexpr int CW = PermCfg<T>::CW;
  extern __shared__ __align__(16) char smem_raw[];
  cplx<T> *buf = reinterpret_cast<cplx<T> *>(smem_raw);  // [nmove][CW]
  __shared__ int psrc[kPlanMax], pdst[kPlanMax];
  const int nmove = min(plan[0], kPlanMax);
  const int n1 = c1 - c0;
  const int ntot = n1 + (c3 - c2);
  const int cbase = blockIdx.x * CW;
  const int tid = threadIdx.x;
  for (int m = tid; m < nmove; m += 256) {
    psrc[m] = plan[1 + kPlanMax + m];
    pdst[m] = plan[1 + m];
  }
  __syncthreads();
  // every source element into LDS before any destination is written (FP32:
  // eight loads per thread in flight; an FP64 batch would go to scratch)
  if constexpr (sizeof(T) == 4) {
    for (int e0 = 0; e0 < nmove * CW; e0 += 8 * 256) {
      cplx<T> v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int e = e0 + u * 256 + tid;
        const int m = e / CW, cc = e - m * CW, t = cbase + cc;
        if (e < nmove * CW && t < ntot) v[u] = A[(long)psrc[m] * lda + ((t < n1) ? c0 + t : c2 + (t - n1))];
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int e = e0 + u * 256 + tid;
        const int m = e / CW, cc = e - m * CW, t = cbase + cc;
        if (e < nmove * CW && t < ntot) buf[e] = v[u];
      }
    }
  } else {
    for (int e = tid; e < nmove * CW; e += 256) {
      const int m = e / CW, cc = e - m * CW, t = cbase + cc;
      if (t < ntot) buf[e] = A[(long)psrc[m] * lda + ((t < n1) ? c0 + t : c2 + (t - n1))];
    }
  }
  __syncthreads();
  for (int e = tid; e < nmove * CW; e += 256) {
    const int m = e / CW, cc = e - m * CW;
    const int t = cbase + cc;
    if (t < ntot) {
      const int col = (t < n1) ? c0 + t : c2 + (t - n1);
      A[(long)pdst[m] * lda + col] = buf[e];
    }
  }
}

template <typename T>
static int laswp(cplx<T> *A, long lda, const int *ipiv, int k0, int k1, int c0, int c1, int c2, int c3,
                 int *perm, int n, int *plan, int *info, hipStream_t st) {
  const int kb = k1 - k0;
  if (kb <= 0) return HP_OK;
  if (kb > kOuterBlock) return HP_ERR_ARG;
  c1 = std::max(c0, c1);
  c3 = std::max(c2, c3);
  const long ntot = (long)(c1 - c0) + (c3 - c2);
  TraceScope ts(TR_LASWP, st, 0.0, 4.0 * kb * ntot * sizeof(cplx<T>));
  hipLaunchKernelGGL(swap_plan_kernel, dim3(1), dim3(256), 0, st, ipiv, k0, kb, n, plan, perm, info);
  HP_CHECK_LAUNCH();
  if (ntot == 0) return HP_OK;
  constexpr int CW = PermCfg<T>::CW;
  const size_t shm = (size_t)2 * kb * CW * sizeof(cplx<T>);
  int rc = ensure_dynamic_lds((const void *)row_permute_kernel<T>, shm);
  if (rc) return rc;
  hipLaunchKernelGGL(row_permute_kernel<T>, dim3((unsigned)((ntot + CW - 1) / CW)), dim3(256), shm, st, A, lda,
                     plan, c0, c1, c2, c3);
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

template <typename T, bool UPPER, int CW>
__global__ __launch_bounds__(256) void trsm_kernel(int m, int ncols, const cplx<T> *__restrict__ L, long ldl,
                                                   cplx<T> *__restrict__ X, long ldx) {
  constexpr int BS = kTrsmBS;
  constexpr int LP = BS + 1;
  extern __shared__ __align__(16) char smem_raw[];
  cplx<T> *Xs = reinterpret_cast<cplx<T> *>(smem_raw);  // [m][CW]
  cplx<T> *Lp = Xs + (size_t)m * CW;                    // [m][LP]: the current 16-column panel of L
  const int tid = threadIdx.x;
  const int col0 = blockIdx.x * CW;
  const int ncw = min(CW, ncols - col0);
  for (int e = tid; e < m * CW; e += 256) {
    const int rr = e / CW, cc = e - rr * CW;
    cplx<T> v{T(0), T(0)};
    if (cc < ncw) v = X[(long)rr * ldx + col0 + cc];
    Xs[e] = v;
  }
  const int nblk = (m + BS - 1) / BS;
  for (int bi = 0; bi < nblk; ++bi) {
    const int b = UPPER ? (nblk - 1 - bi) : bi;
    const int r0 = b * BS;
    const int bs = min(BS, m - r0);
    // rows that read this panel: the diagonal block and the rows still to update
    const int lr0 = UPPER ? 0 : r0;
    const int lr1 = UPPER ? r0 + bs : m;
    for (int e = tid; e < (lr1 - lr0) * BS; e += 256) {
      const int rr = lr0 + e / BS, jj = e % BS;
      cplx<T> v{T(0), T(0)};
      if (jj < bs) v = L[(long)rr * ldl + r0 + jj];
      if (UPPER && rr == r0 + jj) v = crcp(v);  // reciprocal of the diagonal of U
      Lp[rr * LP + jj] = v;
    }
    __syncthreads();
    // diagonal solve: one thread per column
    if (tid < CW) {
      const int cc = tid;
      if (!UPPER) {
        for (int ii = 1; ii < bs; ++ii) {
          cplx<T> sum = Xs[(r0 + ii) * CW + cc];
          for (int jj = 0; jj < ii; ++jj) sum = cfms(sum, Lp[(r0 + ii) * LP + jj], Xs[(r0 + jj) * CW + cc]);
          Xs[(r0 + ii) * CW + cc] = sum;
        }
      } else {
        for (int ii = bs - 1; ii >= 0; --ii) {
          cplx<T> sum = Xs[(r0 + ii) * CW + cc];
          for (int jj = ii + 1; jj < bs; ++jj) sum = cfms(sum, Lp[(r0 + ii) * LP + jj], Xs[(r0 + jj) * CW + cc]);
          Xs[(r0 + ii) * CW + cc] = cmul(sum, Lp[(r0 + ii) * LP + ii]);
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
      cplx<T> sum = Xs[rr * CW + cc];
      const cplx<T> *lrow = Lp + rr * LP;
#pragma unroll 4
      for (int jj = 0; jj < bs; ++jj) sum = cfms(sum, lrow[jj], Xs[(r0 + jj) * CW + cc]);
      Xs[rr * CW + cc] = sum;
    }
    __syncthreads();
  }
  for (int e = tid; e < m * CW; e += 256) {
    const int rr = e / CW, cc = e - rr * CW;
    if (cc < ncw) X[(long)rr * ldx + col0 + cc] = Xs[e];
  }
}

template <typename T, bool UPPER, int CW>
static int trsm_launch(int m, int ncols, const cplx<T> *L, long ldl, cplx<T> *X, long ldx, hipStream_t st) {
  const size_t shm = (size_t)m * (CW + kTrsmBS + 1) * sizeof(cplx<T>);
  int rc = ensure_dynamic_lds((const void *)trsm_kernel<T, UPPER, CW>, shm);
  if (rc) return rc;
  hipLaunchKernelGGL((trsm_kernel<T, UPPER, CW>), dim3((ncols + CW - 1) / CW), dim3(256), shm, st, m, ncols, L,
                     ldl, X, ldx);
  HP_CHECK_LAUNCH();
  return HP_OK;
}

// Narrow column stripes when there are few columns (the solves: n_c
// right-hand sides), wide ones otherwise (the U rows of the factorization).
template <typename T, bool UPPER>
static int trsm(int m, int ncols, const cplx<T> *L, long ldl, cplx<T> *X, long ldx, hipStream_t st) {
  if (m <= 0 || ncols <= 0) return HP_OK;
  if (m > kTrsmMaxRows) return HP_ERR_ARG;
  TraceScope ts(TR_TRSM, st, 4.0 * m * m * (double)ncols, 0.0);
  if (ncols <= 2048) return trsm_launch<T, UPPER, 8>(m, ncols, L, ldl, X, ldx, st);
  return trsm_launch<T, UPPER, TrsmCfg<T>::CW>(m, ncols, L, ldl, X, ldx, st);
}

// --------------------------------------------------------- panel finish --
//
// After the panel of jb <= kPanelWidth columns at j inside the outer block
// [k, kend): the panel's interchanges on the block's other columns ([k, j)
// and [j + jb, kend)) and the panel's U rows U12 = L11^-1 A12 on the columns
// right of it, in one launch.  One workgroup per stripe of CW columns:
//  1. the net row permutation of the jb interchanges, worked out by one
//     wavefront: the jb block rows and the distinct pivot rows below the
//     block are the slots (at most 2 jb); lane s tracks which original row's
//     content sits in slot s while the interchanges are replayed in order;
//  2. every slot's source row of the stripe into LDS (all reads before any
//     write), then the rows that move below the block, and the block rows
//     of the columns left of the panel, written back;
//  3. right of the panel, forward substitution with the panel's unit lower
//     L11 on the block rows (one thread per column: FP32 columns held in
//     registers, FP64 in 8-row register blocks), written back.
template <typename T>
struct FinishCfg {
  static constexpr int CW = 32;  // 2 kPanelWidth x CW must be a multiple of 256
};
template <>
struct FinishCfg<float> {
  static constexpr int CW = 64;
};

template <typename T>
__global__ __launch_bounds__(256) void panel_finish_kernel(int n, int k, int kend, int j, int jb,
                                                           cplx<T> *__restrict__ A, long lda,
                                                           const int *__restrict__ ipiv, int *__restrict__ info) {
  constexpr int CW = FinishCfg<T>::CW;
  constexpr int W = kPanelWidth;
  constexpr int LP = W + 1;
  __builtin_amdgcn_s_setprio(3);  // on the panel chain, like panel_kernel
  extern __shared__ __align__(16) char smem_raw[];
  cplx<T> *buf = reinterpret_cast<cplx<T> *>(smem_raw);  // [2 W][CW]: the stripe's slot contents
  cplx<T> *Lt = buf + 2 * W * CW;                         // [W][LP]: L11
  __shared__ int ps[W], src[2 * W], dst[2 * W];
  __shared__ int nslot;
  const int tid = threadIdx.x;
  const int n1 = j - k;                   // stripe columns left of the panel
  const int ntot = n1 + (kend - j - jb);  // and in total
  const int q0 = blockIdx.x * CW;
  if (tid < jb) {
    int p = ipiv[j + tid];
    if (p < j + tid || p >= n) {  // never expected; keep every index in range
      atomicExch(info, -1);
      p = j + tid;
    }
    ps[tid] = p;
  }
  __syncthreads();
  if (tid < 64) {
    const int lane = tid;
    const int p = lane < jb ? ps[lane] : 0;
    const bool out = lane < jb && p >= j + jb;
    int f = lane;  // first interchange that brings row p in
    for (int i = 0; i < jb; ++i) {
      const int pi = __builtin_amdgcn_readlane(p, i);
      if (out && i < f && pi == p) f = i;
    }
    const unsigned long long firsts = __ballot(out && f == lane);
    const int nout = __popcll(firsts);
    // slot of this lane's pivot row, and the original row of slot `lane`
    const int b = lane < jb ? (out ? jb + __popcll(firsts & ((1ull << f) - 1)) : p - j) : lane;
    int row = lane < jb ? j + lane : -1;
    for (int i = 0; i < jb; ++i) {
      const int pi = __builtin_amdgcn_readlane(p, i);
      if ((firsts >> i) & 1ull)
        if (lane == jb + (int)__popcll(firsts & ((1ull << i) - 1))) row = pi;
    }
    int content = row;
    for (int i = 0; i < jb; ++i) {
      const int bi = __builtin_amdgcn_readlane(b, i);
      const int vi = __builtin_amdgcn_readlane(content, i);
      const int vb = __builtin_amdgcn_readlane(content, bi);
      if (lane == i) content = vb;
      if (lane == bi) content = vi;
    }
    if (lane < jb + nout) {
      src[lane] = content;
      dst[lane] = row;
    }
    if (lane == 0) nslot = jb + nout;
  }
  __syncthreads();
  const int ns = nslot;
  const int ncw = min(CW, ntot - q0);
  const bool right = q0 + ncw > n1;
  if constexpr (sizeof(T) == 4) {
    // every load of the stripe and of L11 in flight before the first LDS store
    constexpr int kGather = 2 * W * CW / 256, kLoadL = W * W / 256;
    cplx<T> gv[kGather], lv[kLoadL];
#pragma unroll
    for (int u = 0; u < kGather; ++u) {
      const int e = tid + 256 * u, sl = e / CW, c = e - sl * CW, q = q0 + c;
      cplx<T> v{T(0), T(0)};
      if (sl < ns && c < ncw) v = A[(long)src[sl] * lda + (q < n1 ? k + q : j + jb + (q - n1))];
      gv[u] = v;
    }
#pragma unroll
    for (int u = 0; u < kLoadL; ++u) {
      const int e = tid + 256 * u, r = e / W, c = e - r * W;
      cplx<T> v{T(0), T(0)};
      if (right && r < jb && c < jb) v = A[(long)(j + r) * lda + j + c];
      lv[u] = v;
    }
#pragma unroll
    for (int u = 0; u < kGather; ++u) {
      const int e = tid + 256 * u, sl = e / CW, c = e - sl * CW;
      if (sl < ns && c < ncw) buf[e] = gv[u];
    }
#pragma unroll
    for (int u = 0; u < kLoadL; ++u) {
      const int e = tid + 256 * u, r = e / W, c = e - r * W;
      Lt[r * LP + c] = lv[u];
    }
  } else {
    if (right)
      for (int e = tid; e < W * W; e += 256) {
        const int r = e / W, c = e - r * W;
        Lt[r * LP + c] = (r < jb && c < jb) ? A[(long)(j + r) * lda + j + c] : cplx<T>{T(0), T(0)};
      }
    for (int e = tid; e < ns * CW; e += 256) {
      const int sl = e / CW, c = e - sl * CW, q = q0 + c;
      if (c < ncw) buf[e] = A[(long)src[sl] * lda + (q < n1 ? k + q : j + jb + (q - n1))];
    }
  }
  __syncthreads();
  for (int e = tid; e < ns * CW; e += 256) {
    const int sl = e / CW, c = e - sl * CW, q = q0 + c;
    if (c < ncw && src[sl] != dst[sl] && (sl >= jb || q < n1))
      A[(long)dst[sl] * lda + (q < n1 ? k + q : j + jb + (q - n1))] = buf[e];
  }
  if (tid < ncw && q0 + tid >= n1) {
    const int col = j + jb + (q0 + tid - n1);
    if constexpr (sizeof(T) == 4) {
      // the column in registers, every index static
      cplx<T> x[W];
#pragma unroll
      for (int i = 0; i < W; ++i) x[i] = i < jb ? buf[i * CW + tid] : cplx<T>{T(0), T(0)};
#pragma unroll
      for (int i = 1; i < W; ++i)
        if (i < jb) {
#pragma unroll
          for (int kk = 0; kk < i; ++kk) x[i] = cfms(x[i], Lt[i * LP + kk], x[kk]);
        }
#pragma unroll
      for (int i = 0; i < W; ++i)
        if (i < jb) A[(long)(j + i) * lda + col] = x[i];
    } else {
      // 8 rows at a time in registers, the rows solved before them read back
      // from LDS (rows past jb meet only zeros of L11 and are never stored)
      constexpr int RB = 8;
#pragma unroll 1
      for (int r0 = 0; r0 < jb; r0 += RB) {
        cplx<T> acc[RB];
#pragma unroll
        for (int i = 0; i < RB; ++i) acc[i] = buf[(r0 + i) * CW + tid];
#pragma unroll 1
        for (int kk = 0; kk < r0; ++kk) {
          const cplx<T> xk = buf[kk * CW + tid];
#pragma unroll
          for (int i = 0; i < RB; ++i) acc[i] = cfms(acc[i], Lt[(r0 + i) * LP + kk], xk);
        }
#pragma unroll
        for (int i = 1; i < RB; ++i)
#pragma unroll
          for (int kk = 0; kk < i; ++kk) acc[i] = cfms(acc[i], Lt[(r0 + i) * LP + r0 + kk], acc[kk]);
#pragma unroll
        for (int i = 0; i < RB; ++i)
          if (r0 + i < jb) {
            buf[(r0 + i) * CW + tid] = acc[i];
            A[(long)(j + r0 + i) * lda + col] = acc[i];
          }
      }
    }
  }
}

template <typename T>
static int panel_finish(int n, int k, int kend, int j, int jb, cplx<T> *A, long lda, const int *ipiv, int *info,
                        hipStream_t st) {
  if (jb <= 0 || jb > kPanelWidth || j < k || j + jb > kend || kend > n) return HP_ERR_ARG;
  const int ntot = (j - k) + (kend - j - jb);
  if (ntot == 0) return HP_OK;
  constexpr int CW = FinishCfg<T>::CW;
  const size_t shm = ((size_t)2 * kPanelWidth * CW + (size_t)kPanelWidth * (kPanelWidth + 1)) * sizeof(cplx<T>);
  int rc = ensure_dynamic_lds((const void *)panel_finish_kernel<T>, shm);
  if (rc) return rc;
  const int nright = kend - j - jb;
  TraceScope ts(TR_TRSM, st, 4.0 * jb * jb * (double)nright, 4.0 * jb * ntot * sizeof(cplx<T>));
  hipLaunchKernelGGL(panel_finish_kernel<T>, dim3((unsigned)((ntot + CW - 1) / CW)), dim3(256), shm, st, n, k, kend,
                     j, jb, A, lda, ipiv, info);
  HP_CHECK_LAUNCH();
  return HP_OK;
}

// ------------------------------------------- inverted diagonal blocks --
// The FP32 factor is applied many times per energy (once per refinement
// step).  Its triangular solves are restructured for that reuse: the
// kInvBlock x kInvBlock diagonal blocks of L and U are inverted once, and each
// block step of a solve becomes a small in-place product with the inverse
// followed by the trailing GEMM, instead of a latency-bound substitution.
// The refinement corrects the slightly larger rounding error of the products.
// FP64 keeps the substitution (its single solve sets the accuracy).
constexpr int kInvLd = kInvBlock + 1;  // LDS row stride (complex elements)

// One workgroup per diagonal block: block index blk0 + blockIdx.x; blockIdx.y
// == 0 inverts the unit-lower block of L, blockIdx.y == 1 the upper block of
// U.  The block is staged in LDS (extended by the identity past a ragged
// edge) and inverted by recursive doubling: first its eight 16 x 16 diagonal
// blocks (one thread per column, substitution in registers), then for
// s = 16, 32, 64 every 2s-block from its two inverted s-blocks,
//   [A 0; C D]^-1 = [A^-1 0; -D^-1 C A^-1  D^-1]   (lower),
//   [A B; 0 D]^-1 = [A^-1  -A^-1 B D^-1; 0 D^-1]   (upper),
// each off-diagonal product formed by all threads in two in-place passes.
// Output: dense kInvBlock x kInvBlock row-major blocks, the nbt lower inverses
// first, then the nbt upper ones; entries outside a ragged last block are zero.
constexpr int kInvBase = 16;
template <typename T>
__global__ __launch_bounds__(256) void tri_inverse_kernel(int n, int blk0, int nbt, const cplx<T> *__restrict__ LU,
                                                          long lda, cplx<T> *__restrict__ Inv) {
  constexpr int NB = kInvBlock, LD = kInvLd, B0 = kInvBase;
  constexpr int ND = NB / B0;  // diagonal base blocks
  extern __shared__ __align__(16) char smem_raw[];
  cplx<T> *X = reinterpret_cast<cplx<T> *>(smem_raw);  // [NB][LD]
  cplx<T> *Dg = X + NB * LD;                           // [ND][B0][B0 + 1]
  const bool upper = blockIdx.y != 0;
  const int blk = blk0 + blockIdx.x;
  const int b0 = blk * NB;
  const int bs = min(NB, n - b0);
  const cplx<T> *Tb = LU + (long)b0 * lda + b0;
  const int tid = threadIdx.x;
  const cplx<T> zero{T(0), T(0)};
  // stage the triangle (strict lower of L, upper of U incl. its diagonal)
  for (int e0 = 0; e0 < NB * NB; e0 += 8 * 256) {
    cplx<T> v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {  // all loads first (clamped addresses), then the masks
      const int e = e0 + u * 256 + tid;
      const int r = e / NB, c = e - r * NB;
      v[u] = Tb[(long)min(r, bs - 1) * lda + min(c, bs - 1)];
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = e0 + u * 256 + tid;
      const int r = e / NB, c = e - r * NB;
      const bool in = r < bs && c < bs && (upper ? (r <= c) : (r > c));
      cplx<T> x = in ? v[u] : zero;
      if (!(r < bs && c < bs) && r == c) x.re = T(1);
      X[r * LD + c] = x;
    }
  }
  __syncthreads();
  // inverses of the diagonal 16 x 16 blocks: thread (d, jj) solves for column jj of block d
  if (tid < ND * B0) {
    const int d = tid / B0, jj = tid - d * B0, o = d * B0;
    cplx<T> x[B0];
    if (!upper) {
#pragma unroll
      for (int ii = 0; ii < B0; ++ii) {
        cplx<T> acc{T(ii == jj ? 1 : 0), T(0)};
#pragma unroll
        for (int k = 0; k < ii; ++k) acc = cfms(acc, X[(o + ii) * LD + o + k], x[k]);
        x[ii] = acc;
      }
    } else {
#pragma unroll
      for (int ii = B0 - 1; ii >= 0; --ii) {
        cplx<T> acc{T(ii == jj ? 1 : 0), T(0)};
#pragma unroll
        for (int k = ii + 1; k < B0; ++k) acc = cfms(acc, X[(o + ii) * LD + o + k], x[k]);
        x[ii] = cmul(acc, crcp(X[(o + ii) * LD + o + ii]));
      }
    }
#pragma unroll
    for (int ii = 0; ii < B0; ++ii) Dg[(d * B0 + ii) * (B0 + 1) + jj] = x[ii];
  }
  __syncthreads();
  for (int e = tid; e < ND * B0 * B0; e += 256) {
    const int d = e / (B0 * B0), ii = (e / B0) % B0, jj = e % B0;
    X[(d * B0 + ii) * LD + d * B0 + jj] = Dg[(d * B0 + ii) * (B0 + 1) + jj];
  }
  __syncthreads();
  // doubling: level s combines pairs of inverted s-blocks
  for (int s = B0; s < NB; s *= 2) {
    const int per = (NB / 2) * s / 256;  // elements per thread: 4, 8, 16
    cplx<T> t[NB / 8];
    // pass 1: T = C A (lower) or T = B D (upper), into registers
#pragma unroll
    for (int q = 0; q < NB / 8; ++q) {
      if (q >= per) break;
      const int e = tid + 256 * q;
      const int p = e / (s * s), rem = e - p * s * s, r = rem / s, c = rem - r * s, o = 2 * s * p;
      cplx<T> acc = zero;
      if (!upper) {
        for (int k = c; k < s; ++k) acc = cfms(acc, X[(o + s + r) * LD + o + k], X[(o + k) * LD + o + c]);
      } else {
        for (int k = 0; k <= c; ++k) acc = cfms(acc, X[(o + r) * LD + o + s + k], X[(o + s + k) * LD + o + s + c]);
      }
      t[q] = acc;  // holds -T
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < NB / 8; ++q) {
      if (q >= per) break;
      const int e = tid + 256 * q;
      const int p = e / (s * s), rem = e - p * s * s, r = rem / s, c = rem - r * s, o = 2 * s * p;
      if (!upper)
        X[(o + s + r) * LD + o + c] = t[q];
      else
        X[(o + r) * LD + o + s + c] = t[q];
    }
    __syncthreads();
    // pass 2: D^-1 (-T) (lower) or A^-1 (-T) (upper), in place of T
#pragma unroll
    for (int q = 0; q < NB / 8; ++q) {
      if (q >= per) break;
      const int e = tid + 256 * q;
      const int p = e / (s * s), rem = e - p * s * s, r = rem / s, c = rem - r * s, o = 2 * s * p;
      cplx<T> acc = zero;
      if (!upper) {
        for (int k = 0; k <= r; ++k) {
          const cplx<T> a = X[(o + s + r) * LD + o + s + k], b = X[(o + s + k) * LD + o + c];
          acc.re += a.re * b.re - a.im * b.im;
          acc.im += a.re * b.im + a.im * b.re;
        }
      } else {
        for (int k = r; k < s; ++k) {
          const cplx<T> a = X[(o + r) * LD + o + k], b = X[(o + k) * LD + o + s + c];
          acc.re += a.re * b.re - a.im * b.im;
          acc.im += a.re * b.im + a.im * b.re;
        }
      }
      t[q] = acc;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < NB / 8; ++q) {
      if (q >= per) break;
      const int e = tid + 256 * q;
      const int p = e / (s * s), rem = e - p * s * s, r = rem / s, c = rem - r * s, o = 2 * s * p;
      if (!upper)
        X[(o + s + r) * LD + o + c] = t[q];
      else
        X[(o + r) * LD + o + s + c] = t[q];
    }
    __syncthreads();
  }
  cplx<T> *out = Inv + ((size_t)blockIdx.y * nbt + blk) * NB * NB;
  for (int e = tid; e < NB * NB; e += 256) {
    const int r = e / NB, c = e - r * NB;
    cplx<T> v = zero;
    if (r < bs && c < bs) v = X[r * LD + c];
    out[e] = v;
  }
}

// Inverts diagonal blocks [blk0, blk0 + nblk) of L (and of U when `both`).
template <typename T>
static int tri_inverse(int n, const cplx<T> *LU, long lda, cplx<T> *inv, int blk0, int nblk, bool both,
                       hipStream_t st) {
  if (nblk <= 0) return HP_OK;
  const size_t shm = ((size_t)kInvBlock * kInvLd + (size_t)kInvBlock * (kInvBase + 1)) * sizeof(cplx<T>);
  int rc = ensure_dynamic_lds((const void *)tri_inverse_kernel<T>, shm);
  if (rc) return rc;
  const int nbt = (n + kInvBlock - 1) / kInvBlock;
  TraceScope ts(TR_TRSM, st, (both ? 2.0 : 1.0) * (8.0 / 6.0) * (double)kInvBlock * kInvBlock * kInvBlock * nblk,
                0.0);
  hipLaunchKernelGGL(tri_inverse_kernel<T>, dim3(nblk, both ? 2 : 1), dim3(256), shm, st, n, blk0, nbt, LU, lda,
                     inv);
  HP_CHECK_LAUNCH();
  return HP_OK;
}

size_t inverse_bytes(int n, int prec) {
  if (!is_c64(prec)) return 0;
  const size_t nb = (size_t)(n + kInvBlock - 1) / kInvBlock;
  return 2 * nb * kInvBlock * kInvBlock * sizeof(cplx<float>);
}

// LDS row stride of a staged 128 x 128 inverse (diag256_kernel): keeps rows
// 16-byte aligned and spreads the banks.
constexpr int kApplyLd = kInvBlock + 2;

// ------------------------------------------------------------ factorization --

template <typename T>
struct PanelSlots {
  cplx<T> *rows;  // [2][G][W]
  T *val;         // [2][G]
  int *row;       // [2][G]
  cplx<T> *diag;  // [2][W]
  unsigned long long *key;  // [2][G] (FP32 panels)
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
  off += align_up(sizeof(cplx<T>) * 2 * kPanelWidth, 256);
  s.key = (unsigned long long *)(base + off);
  return s;
}

static size_t slot_bytes_max() {
  return align_up(sizeof(cplx<double>) * 2 * kMaxPanelGroups * kPanelWidth, 256) +
         align_up(sizeof(double) * 2 * kMaxPanelGroups, 256) + align_up(sizeof(int) * 2 * kMaxPanelGroups, 256) +
         align_up(sizeof(cplx<double>) * 2 * kPanelWidth, 256) +
         align_up(sizeof(unsigned long long) * 2 * kMaxPanelGroups, 256);
}
static size_t slot_key_words() { return 2 * 2 * kMaxPanelGroups; }  // 32-bit words of PanelSlots::key

// Rows per workgroup of the panel grid, and the grid size.
// Number of factorizations that may run at the same time on one device
// (hp_set_concurrency).
std::atomic<int> g_concurrency{1};


template <typename T>
static int panel_grid(int m, int lds_cap, int &G, int &rpw) {
  // at least 64 rows per workgroup, at most kMaxPanelGroups workgroups (one
  // per CU; a 25600-row panel: 128 groups factor ~9% faster than 64 with the
  // per-group arrival flags), and at most lds_cap bytes of rows per workgroup
  const int rpw_max = lds_cap / (int)(kPanelLd * sizeof(cplx<T>));
  const int rpw_min = 64;
  // FP32: 128 workgroups (measured fastest on a 25600-row panel); FP64: up to
  // 256 (at most 53 KB of rows each at 25600 rows), so that a panel
  // workgroup fits beside the FP64 trailing update's workgroups on a CU
  static const int gmax64 = [] {
    const char *e = getenv("HP_PANEL_GMAX64");
    const int v = e ? atoi(e) : kMaxPanelGroups;
    return std::max(1, std::min(v, kMaxPanelGroups));
  }();
  const int gmax = std::is_same<T, double>::value ? gmax64 : 128;
  G = (m + rpw_min - 1) / rpw_min;
  G = std::min(G, gmax);
  G = std::max(G, 1);
  // tuning knob: HP_PANEL_GROUPS overrides the workgroup count (still capped by LDS below)
  static const int forced = [] {
    const char *e = getenv("HP_PANEL_GROUPS");
    return e ? atoi(e) : 0;
  }();
  if (forced > 0) G = std::min(forced, kMaxPanelGroups);
  rpw = (m + G - 1) / G;
  if (rpw > rpw_max) {
    rpw = rpw_max;
    G = (m + rpw - 1) / rpw;
    if (G > kMaxPanelGroups) return HP_ERR_UNSUPPORTED;  // the rows do not fit the workgroups' LDS
  }
  return HP_OK;
}

static int device_cus(int *cus) {
  int dev = 0;
  HP_CHECK_HIP(hipGetDevice(&dev));
  HP_CHECK_HIP(hipDeviceGetAttribute(cus, hipDeviceAttributeMultiprocessorCount, dev));
  return HP_OK;
}

template <typename T>
static int panel(int n, int j0, int w, cplx<T> *A, long lda, int *ipiv, int *info, unsigned *bar,
                 const PanelSlots<T> &s, hipStream_t st) {
  const int m = n - j0;
  int cus = 0, G, rpw;
  int rc0 = device_cus(&cus);
  if (rc0) return rc0;
  // with other streams' work on the device, small workgroups (64 KB of rows,
  // or just what a grid of kMaxPanelGroups needs when that is more) so that
  // each finds room beside the kernels already resident
  const int conc = g_concurrency.load(std::memory_order_relaxed);
  const int rows_needed = (m + kMaxPanelGroups - 1) / kMaxPanelGroups;
  const int small_cap = std::max(64 * 1024, rows_needed * kPanelLd * (int)sizeof(cplx<T>));
  if ((rc0 = panel_grid<T>(m, conc > 1 ? std::min(small_cap, 150 * 1024) : 150 * 1024, G, rpw))) return rc0;
  if (G > kMaxPanelGroups || G > cus) return HP_ERR_UNSUPPORTED;
  // the FP32 key word holds the row offset and the column epoch in 32 bits
  if (std::is_same<T, float>::value && (rpw >= (int)kKeyNoRow || n >= kKeyMaxColumns)) return HP_ERR_UNSUPPORTED;
  size_t shm = (size_t)rpw * kPanelLd * sizeof(cplx<T>);
  int rc = ensure_dynamic_lds((const void *)panel_kernel<T>, shm);
  if (rc) return rc;
  int nn = n, jj0 = j0, ww = w, rp = rpw;
  long ld = lda;
  cplx<T> *srows = s.rows;
  T *sval = s.val;
  int *srow = s.row;
  cplx<T> *sdiag = s.diag;
  unsigned long long *skey = s.key;
  void *args[] = {&nn, &jj0, &ww, &A, &ld, &ipiv, &info, &bar, &srows, &sval, &srow, &sdiag, &skey, &rp};
  // All G workgroups must become resident together (they meet at grid
  // barriers).  G is at most one per CU and one workgroup fits a CU, so on an
  // idle device they are; beside other kernels (this factorization's own
  // trailing update, other streams' work) they become resident as those
  // kernels' workgroups retire, which the barriers' bounded waits cover.
  // Only one factorization's panels are on the device at any time (see
  // lu_factor), so panel grids never wait for each other.
  TraceScope ts(TR_PANEL, st, 4.0 * (double)m * w * w, 2.0 * sizeof(cplx<T>) * (double)m * w);
  HP_CHECK_HIP(hipLaunchKernel((const void *)panel_kernel<T>, dim3(G), dim3(256), args, shm, st));
  return HP_OK;
}

// Second stream and events for the look-ahead, one set per (device, caller
// stream), created on first use (default priority).  A factorization holds
// its set's lock while it enqueues, so two host threads that factor on one
// stream serialize, and factorizations on different streams overlap.
namespace {
struct LookAhead {
  std::mutex mu;
  hipStream_t panel = nullptr;
  hipEvent_t ready = nullptr, done = nullptr;
};
std::mutex g_la_mu;
std::map<std::pair<int, hipStream_t>, std::unique_ptr<LookAhead>> g_la;

int lookahead_for(hipStream_t st, LookAhead **out) {
  int dev = 0;
  HP_CHECK_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_la_mu);
  std::unique_ptr<LookAhead> &la = g_la[{dev, st}];
  if (!la) {
    auto fresh = std::make_unique<LookAhead>();
    HP_CHECK_HIP(hipStreamCreateWithFlags(&fresh->panel, hipStreamNonBlocking));
    HP_CHECK_HIP(hipEventCreateWithFlags(&fresh->ready, hipEventDisableTiming));
    HP_CHECK_HIP(hipEventCreateWithFlags(&fresh->done, hipEventDisableTiming));
    la = std::move(fresh);
  }
  *out = la.get();
  return HP_OK;
}
}  // namespace

// Factors the columns [k, k + kb) of the rows below k: kPanelWidth-wide
// panels, each followed by its interchanges on the block's other columns and
// by the update of the block's columns to its right.
template <typename T>
static int factor_block(int n, int k, int kb, cplx<T> *A, long lda, int *ipiv, int *info, unsigned *bars,
                        const PanelSlots<T> &slots, hipStream_t st) {
  int rc;
  const size_t per_panel = barrier_words(kMaxPanelGroups);
  for (int j = k; j < k + kb; j += kPanelWidth) {
    const int jb = std::min(kPanelWidth, k + kb - j);
    if ((rc = panel<T>(n, j, jb, A, lda, ipiv, info, bars + per_panel * (j / kPanelWidth), slots, st)))
      return rc;
    // the panel's interchanges on the block's other columns, and its U rows
    if ((rc = panel_finish<T>(n, k, k + kb, j, jb, A, lda, ipiv, info, st))) return rc;
    const int rest = k + kb - (j + jb);
    if (rest > 0) {
      cplx<T> *A12 = A + (long)j * lda + j + jb;
      if ((rc = gemm_sub<T>(n - j - jb, rest, jb, A + (long)(j + jb) * lda + j, lda, A12, lda,
                            A + (long)(j + jb) * lda + j + jb, lda, st)))
        return rc;
    }
  }
  return HP_OK;
}

// Inverts the two 128-row diagonal blocks of L11 of the (factored) block at
// k into the workspace (FP32 only; FP64 substitutes).
template <typename T>
static int invert_block(int n, int k, const cplx<T> *A, long lda, char *work, const Workspace &ws,
                        hipStream_t st) {
  if constexpr (std::is_same<T, float>::value)
    return tri_inverse<T>(n, A, lda, (cplx<T> *)(work + ws.inv_off), k / kInvBlock, 2, false, st);
  (void)n, (void)k, (void)A, (void)lda, (void)work, (void)ws, (void)st;
  return HP_OK;
}

template <typename T>
__global__ void copy_rows_kernel(int n, int nrhs, const cplx<T> *__restrict__ X, long ldx, cplx<T> *__restrict__ Y,
                                 long ldy);

// U12 = L11^-1 A12 for the kb rows of block k and the ncols columns right of
// it (FP32: through the inverses invert_block made).
template <typename T>
static int block_row_solve(int n, int k, int kb, int ncols, cplx<T> *A, long lda, char *work, const Workspace &ws,
                           hipStream_t st) {
  int rc;
  cplx<T> *L11 = A + (long)k * lda + k;
  cplx<T> *A12 = A + (long)k * lda + k + kb;
  if constexpr (std::is_same<T, float>::value) {
    // through the two inverted 128-row diagonal blocks of L11 (kb == 2
    // kInvBlock whenever columns remain)
    static_assert(kOuterBlock == 2 * kInvBlock, "outer block = two inverted blocks");
    if (kb != 2 * kInvBlock) return HP_ERR_ARG;
    cplx<T> *inv = (cplx<T> *)(work + ws.inv_off);
    const int b = k / kInvBlock;
    const size_t iblk = (size_t)kInvBlock * kInvBlock;
    cplx<T> *A22 = A12 + (long)kInvBlock * lda;
    (void)n;
    // each inverse applied as an MFMA product into scratch, then copied back
    // (a product cannot run in place: every output tile reads its whole
    // column panel)
    cplx<T> *tmp = (cplx<T> *)(work + ws.u12_off);
    const long cnt = (long)kInvBlock * ncols;
    const dim3 cgrid((unsigned)((cnt + 255) / 256));
    if ((rc = gemm_set_batched<T>(kInvBlock, ncols, kInvBlock, T(1), inv + b * iblk, kInvBlock, 0, A12, lda, 0, tmp,
                                  ncols, 0, 1, st)))
      return rc;
    hipLaunchKernelGGL(copy_rows_kernel<T>, cgrid, dim3(256), 0, st, kInvBlock, ncols, tmp, (long)ncols, A12, lda);
    HP_CHECK_LAUNCH();
    if ((rc = gemm_sub<T>(kInvBlock, ncols, kInvBlock, L11 + (long)kInvBlock * lda, lda, A12, lda, A22, lda, st)))
      return rc;
    if ((rc = gemm_set_batched<T>(kInvBlock, ncols, kInvBlock, T(1), inv + (b + 1) * iblk, kInvBlock, 0, A22, lda, 0,
                                  tmp, ncols, 0, 1, st)))
      return rc;
    hipLaunchKernelGGL(copy_rows_kernel<T>, cgrid, dim3(256), 0, st, kInvBlock, ncols, tmp, (long)ncols, A22, lda);
    HP_CHECK_LAUNCH();
    return HP_OK;
  } else {
    (void)n;
    (void)work;
    (void)ws;
    // blocked substitution: each 32-row diagonal block of L11 solved in
    // place, the rows below it then updated by an MFMA product (one long
    // substitution over 256 rows is latency-bound and sits on the
    // factorization's critical path)
    constexpr int kSub = kPanelWidth;
    for (int i0 = 0; i0 < kb; i0 += kSub) {
      const int ib = std::min(kSub, kb - i0);
      cplx<T> *Xi = A12 + (long)i0 * lda;
      if ((rc = trsm<T, false>(ib, ncols, L11 + (long)i0 * lda + i0, lda, Xi, lda, st))) return rc;
      if (i0 + ib < kb && (rc = gemm_sub<T>(kb - i0 - ib, ncols, ib, L11 + (long)(i0 + ib) * lda + i0, lda, Xi, lda,
                                            Xi + (long)ib * lda, lda, st)))
        return rc;
    }
    return HP_OK;
  }
}

// Blocked right-looking LU with a one-block look-ahead: once the columns of
// block k+1 have received the update from block k, block k+1 is factored on a
// second stream while the rest of the trailing matrix is updated on the
// caller's stream; the two meet before block k+1's interchanges are applied
// to the other columns.  The panel's latency-bound column steps thus run under
// the MFMA-bound update.
template <typename T>
static int lu_factor_on(int n, cplx<T> *A, long lda, int *ipiv, int *perm, int *info, char *work,
                        const Workspace &ws, hipStream_t st) {
  int rc;
  // the look-ahead stream is needed (and created on first use) only when a
  // block is factored beside a trailing update, i.e. for n > 2 kOuterBlock
  LookAhead *la = nullptr;
  std::unique_lock<std::mutex> lk;
  if (n > 2 * kOuterBlock) {
    if ((rc = lookahead_for(st, &la))) return rc;
    lk = std::unique_lock<std::mutex>(la->mu);
  }
  unsigned *bars = (unsigned *)(work + ws.sync_off);
  const size_t per_panel = barrier_words(kMaxPanelGroups);
  const int npanels = (n + kPanelWidth - 1) / kPanelWidth;
  if ((rc = fill_u32(bars, per_panel * npanels, 0u, st))) return rc;
  if ((rc = fill_u32((unsigned *)info, 1, 0u, st))) return rc;
  hipLaunchKernelGGL(iota_kernel, dim3((n + 255) / 256), dim3(256), 0, st, perm, n);
  HP_CHECK_LAUNCH();
  PanelSlots<T> slots = carve_slots<T>(work + ws.slot_off);
  // key words from an earlier factorization must not match this one's epochs
  if ((rc = fill_u32((unsigned *)slots.key, slot_key_words(), 0u, st))) return rc;
  int *plan = (int *)(work + ws.slot_off + slot_bytes_max());
  if ((rc = factor_block<T>(n, 0, std::min(kOuterBlock, n), A, lda, ipiv, info, bars, slots, st))) return rc;
  for (int k = 0; k < n; k += kOuterBlock) {
    const int kb = std::min(kOuterBlock, n - k);
    // the block's interchanges on all columns outside the block, and on perm
    if ((rc = laswp<T>(A, lda, ipiv, k, k + kb, 0, k, k + kb, n, perm, n, plan, info, st))) return rc;
    const int rest = n - k - kb;
    if (rest <= 0) break;
    const int k2 = k + kb;
    const int kb2 = std::min(kOuterBlock, rest);
    cplx<T> *L21 = A + (long)k2 * lda + k;
    cplx<T> *U12 = A + (long)k * lda + k2;
    cplx<T> *A22 = A + (long)k2 * lda + k2;
    // L11's diagonal blocks inverted on this stream: beside the trailing
    // update, the inversion's whole-CU LDS footprint waits for GEMM
    // workgroups to drain (10x slower there than here)
    if ((rc = invert_block<T>(n, k, A, lda, work, ws, st))) return rc;
    if ((rc = block_row_solve<T>(n, k, kb, rest, A, lda, work, ws, st))) return rc;
    // trailing update A22 -= L21 U12 (the columns [c0, c0 + nc) of it): FP32
    // or FP64 matrix cores, or with HP_C64H the split-FP16 operands made
    // once per block from L21 and U12
    bool h3 = false;
    if constexpr (std::is_same<T, float>::value) h3 = ws.h3 && kb == kOuterBlock;
    auto update = [&](int c0, int ncols) -> int {
      if constexpr (std::is_same<T, float>::value) {
        if (h3)
          return gemm_h3_sub(rest, ncols, kb, work + ws.h3a_off, rest, 0, work + ws.h3b_off, rest, c0, A22 + c0, lda,
                             st);
      }
      return gemm_sub<T>(rest, ncols, kb, L21, lda, U12 + c0, lda, A22 + c0, lda, st);
    };
    if constexpr (std::is_same<T, float>::value) {
      if (h3) {
        if ((rc = h3_convert_rows(rest, kb, L21, lda, work + ws.h3a_off, st))) return rc;
        if ((rc = h3_convert_cols(rest, kb, U12, lda, work + ws.h3b_off, st))) return rc;
      }
    }
    // the next block's columns first
    if ((rc = update(0, kb2))) return rc;
    if (rest > kb2) {  // here n > 2 kOuterBlock, so la is set
      HP_CHECK_HIP(hipEventRecord(la->ready, st));
      HP_CHECK_HIP(hipStreamWaitEvent(la->panel, la->ready, 0));
      if ((rc = factor_block<T>(n, k2, kb2, A, lda, ipiv, info, bars, slots, la->panel))) return rc;
      HP_CHECK_HIP(hipEventRecord(la->done, la->panel));
      if ((rc = update(kb2, rest - kb2))) return rc;
      HP_CHECK_HIP(hipStreamWaitEvent(st, la->done, 0));
    } else {
      if ((rc = factor_block<T>(n, k2, kb2, A, lda, ipiv, info, bars, slots, st))) return rc;
    }
  }
  return HP_OK;
}

// Several factorizations may be requested at once on different streams
// (hp_set_concurrency > 1).  Their panel grids must not wait for each other,
// so they are serialized on one device-wide factorization stream: the
// caller's stream hands over with an event and waits for the result; the
// caller's other work (assembly, solves of other systems) still overlaps.
namespace {
struct FactorQueue {
  std::mutex mu;
  hipStream_t st = nullptr;
  hipEvent_t in = nullptr, out = nullptr;
};
std::mutex g_fq_mu;
std::map<int, std::unique_ptr<FactorQueue>> g_fq;

int factor_queue(FactorQueue **out) {
  int dev = 0;
  HP_CHECK_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_fq_mu);
  std::unique_ptr<FactorQueue> &fq = g_fq[dev];
  if (!fq) {
    auto fresh = std::make_unique<FactorQueue>();
    HP_CHECK_HIP(hipStreamCreateWithFlags(&fresh->st, hipStreamNonBlocking));
    HP_CHECK_HIP(hipEventCreateWithFlags(&fresh->in, hipEventDisableTiming));
    HP_CHECK_HIP(hipEventCreateWithFlags(&fresh->out, hipEventDisableTiming));
    fq = std::move(fresh);
  }
  *out = fq.get();
  return HP_OK;
}
}  // namespace

template <typename T>
int lu_factor(int n, cplx<T> *A, long lda, int *ipiv, int *perm, int *info, char *work, const Workspace &ws,
              hipStream_t st) {
  // a factorization of one block (n <= kOuterBlock: a panel grid of at most
  // four workgroups) runs on the caller's stream in either mode
  if (g_concurrency.load(std::memory_order_relaxed) <= 1 || n <= kOuterBlock)
    return lu_factor_on<T>(n, A, lda, ipiv, perm, info, work, ws, st);
  FactorQueue *fq = nullptr;
  int rc = factor_queue(&fq);
  if (rc) return rc;
  std::lock_guard<std::mutex> lk(fq->mu);
  HP_CHECK_HIP(hipEventRecord(fq->in, st));
  HP_CHECK_HIP(hipStreamWaitEvent(fq->st, fq->in, 0));
  rc = lu_factor_on<T>(n, A, lda, ipiv, perm, info, work, ws, fq->st);
  HP_CHECK_HIP(hipEventRecord(fq->out, fq->st));
  HP_CHECK_HIP(hipStreamWaitEvent(st, fq->out, 0));
  return rc;
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

// Rows per trailing GEMM of the solves: two inverted diagonal blocks (K = 256
// runs the GEMM ~20 % faster than K = 128 on the n_c right-hand sides).
// A 256-row diagonal block of a solve in one launch.  With the first 128-row
// sub-block f and the second s (forward: f above s; backward: f below s):
//   Y_f <- Inv_f Y_f;   Y_s -= M Y_f;   Y_s <- Inv_s Y_s,
// M the off-diagonal block of L (forward) or U (backward), bsec x bf.  A
// workgroup owns a stripe of CW right-hand columns (both sub-blocks in LDS);
// each 128 x 128 operand is staged whole in LDS in turn.  Every staging
// issues all of a thread's loads (in-bounds addresses, out-of-range values
// replaced by zero afterwards) before its first LDS store, so the loads are
// in flight together.

template <typename T>
__device__ __forceinline__ void stage_block(cplx<T> *__restrict__ S, const uint4 *__restrict__ src, int tid) {
  constexpr int EPV = 16 / sizeof(cplx<T>);
  constexpr int NV = kInvBlock * kInvBlock / EPV / 256;
  uint4 buf[NV];
#pragma unroll
  for (int u = 0; u < NV; ++u) buf[u] = src[u * 256 + tid];
#pragma unroll
  for (int u = 0; u < NV; ++u) {
    const int e = (u * 256 + tid) * EPV;
    const int r = e / kInvBlock, k = e - r * kInvBlock;
    *reinterpret_cast<uint4 *>(S + r * kApplyLd + k) = buf[u];
  }
}

template <typename T, int CW>
__global__ __launch_bounds__(256) void diag256_kernel(int bf, int bsec, const cplx<T> *__restrict__ invf,
                                                      const cplx<T> *__restrict__ M, long ldm,
                                                      const cplx<T> *__restrict__ invs, cplx<T> *__restrict__ Yf,
                                                      cplx<T> *__restrict__ Ysec, long ldy, int ncols) {
  constexpr int RPT = kInvBlock * CW / 256;
  constexpr int RSTEP = 256 / CW;
  constexpr int NE = kInvBlock * kInvBlock / 256;  // elements of M per thread
  constexpr int MB = 16;                           // M loads in flight per batch
  static_assert(NE % MB == 0, "staging loop");
  extern __shared__ __align__(16) char smem_raw[];
  cplx<T> *__restrict__ S = reinterpret_cast<cplx<T> *>(smem_raw);  // [kInvBlock][kApplyLd]
  cplx<T> *__restrict__ Fs = S + kInvBlock * kApplyLd;               // [kInvBlock][CW]
  cplx<T> *__restrict__ Ss = Fs + kInvBlock * CW;                     // [kInvBlock][CW]
  const int tid = threadIdx.x;
  const int c = tid % CW, r0 = tid / CW;
  const int col0 = blockIdx.x * CW;
  const bool colok = col0 + c < ncols;
  const int gc = min(col0 + c, ncols - 1);
  const cplx<T> zero{T(0), T(0)};
  {
    cplx<T> vf[RPT], vs[RPT];
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      const int r = r0 + q * RSTEP;
      vf[q] = Yf[(long)min(r, bf - 1) * ldy + gc];
      vs[q] = bsec > 0 ? Ysec[(long)min(r, bsec - 1) * ldy + gc] : zero;
    }
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      const int r = r0 + q * RSTEP;
      Fs[r * CW + c] = (r < bf && colok) ? vf[q] : zero;
      Ss[r * CW + c] = (r < bsec && colok) ? vs[q] : zero;
    }
  }
  cplx<T> acc[RPT];
  auto product = [&](const cplx<T> *__restrict__ Y, int kmax) {
#pragma unroll
    for (int q = 0; q < RPT; ++q) acc[q] = zero;
#pragma unroll 4
    for (int k = 0; k < kmax; ++k) {
      const cplx<T> y = Y[k * CW + c];
#pragma unroll
      for (int q = 0; q < RPT; ++q) {
        const cplx<T> a = S[(r0 + q * RSTEP) * kApplyLd + k];
        acc[q].re += a.re * y.re - a.im * y.im;
        acc[q].im += a.re * y.im + a.im * y.re;
      }
    }
  };
  stage_block<T>(S, reinterpret_cast<const uint4 *>(invf), tid);
  __syncthreads();
  product(Fs, bf);
  __syncthreads();
  for (int q = 0; q < RPT; ++q) Fs[(r0 + q * RSTEP) * CW + c] = acc[q];
  if (bsec > 0) {
    // M (bsec x bf) with 8-byte loads: its rows need not be 16-byte aligned
    for (int e0 = 0; e0 < NE; e0 += MB) {
      cplx<T> buf[MB];
#pragma unroll
      for (int u = 0; u < MB; ++u) {
        const int e = (e0 + u) * 256 + tid;
        const int r = e / kInvBlock, k = e - r * kInvBlock;
        buf[u] = M[(long)min(r, bsec - 1) * ldm + min(k, bf - 1)];
      }
#pragma unroll
      for (int u = 0; u < MB; ++u) {
        const int e = (e0 + u) * 256 + tid;
        const int r = e / kInvBlock, k = e - r * kInvBlock;
        S[r * kApplyLd + k] = (r < bsec && k < bf) ? buf[u] : zero;
      }
    }
    __syncthreads();
    product(Fs, bf);
    __syncthreads();
    for (int q = 0; q < RPT; ++q) {
      const int r = r0 + q * RSTEP;
      const cplx<T> v = Ss[r * CW + c];
      Ss[r * CW + c] = cplx<T>{v.re - acc[q].re, v.im - acc[q].im};
    }
    stage_block<T>(S, reinterpret_cast<const uint4 *>(invs), tid);
    __syncthreads();
    product(Ss, bsec);
    __syncthreads();
    for (int q = 0; q < RPT; ++q) Ss[(r0 + q * RSTEP) * CW + c] = acc[q];
  }
  __syncthreads();
  if (!colok) return;
  for (int q = 0; q < RPT; ++q) {
    const int r = r0 + q * RSTEP;
    if (r < bf) Yf[(long)r * ldy + col0 + c] = Fs[r * CW + c];
    if (r < bsec) Ysec[(long)r * ldy + col0 + c] = Ss[r * CW + c];
  }
}

template <typename T>
static int diag256(int bf, int bsec, const cplx<T> *invf, const cplx<T> *M, long ldm, const cplx<T> *invs,
                   cplx<T> *Yf, cplx<T> *Ysec, long ldy, int ncols, hipStream_t st) {
  // two columns per workgroup: 128 workgroups for 256 right-hand sides,
  // one output row per thread (22 us per launch on MI355X against 35 us with
  // eight columns, whose four dependent rows per thread lengthen each phase)
  constexpr int CW = 2;
  const size_t shm = ((size_t)kInvBlock * kApplyLd + (size_t)2 * kInvBlock * CW) * sizeof(cplx<T>);
  int rc = ensure_dynamic_lds((const void *)diag256_kernel<T, CW>, shm);
  if (rc) return rc;
  TraceScope ts(TR_TRSM, st, 8.0 * ((double)bf * bf + (double)bsec * bf + (double)bsec * bsec) * ncols, 0.0);
  hipLaunchKernelGGL((diag256_kernel<T, CW>), dim3((ncols + CW - 1) / CW), dim3(256), shm, st, bf, bsec, invf, M,
                     ldm, invs, Yf, Ysec, ldy, ncols);
  HP_CHECK_LAUNCH();
  return HP_OK;
}

constexpr int kSolveBlock = 2 * kInvBlock;
static_assert(kSolveBlock <= kTrsmMaxRows, "substitution handles a whole solve block");

// Rows [b, b + bs) of L Y = P B, once the rows above have been eliminated.
template <typename T>
static int diag_forward(int n, int b, int bs, int nrhs, const cplx<T> *LU, long lda, cplx<T> *Y, long ldy,
                        const cplx<T> *inv, hipStream_t st) {
  if (!inv) return trsm<T, false>(bs, nrhs, LU + (long)b * lda + b, lda, Y + (long)b * ldy, ldy, st);
  (void)n;
  const size_t iblk = (size_t)kInvBlock * kInvBlock;
  const int bi = b / kInvBlock, b1 = std::min(kInvBlock, bs), b2 = bs - b1;
  return diag256<T>(b1, std::max(b2, 0), inv + bi * iblk, LU + (long)(b + b1) * lda + b, lda,
                    inv + (bi + 1) * iblk, Y + (long)b * ldy, Y + (long)(b + b1) * ldy, ldy, nrhs, st);
}

// Rows [b, b + bs) of U X = Y, once the rows below have been substituted.
template <typename T>
static int diag_backward(int n, int b, int bs, int nrhs, const cplx<T> *LU, long lda, cplx<T> *Y, long ldy,
                         const cplx<T> *inv, hipStream_t st) {
  if (!inv) return trsm<T, true>(bs, nrhs, LU + (long)b * lda + b, lda, Y + (long)b * ldy, ldy, st);
  const size_t iblk = (size_t)kInvBlock * kInvBlock;
  const int nbt = (n + kInvBlock - 1) / kInvBlock;  // upper inverses follow the lower ones
  const int bi = b / kInvBlock, b1 = std::min(kInvBlock, bs), b2 = bs - b1;
  if (b2 <= 0)
    return diag256<T>(b1, 0, inv + (nbt + bi) * iblk, nullptr, 0, nullptr, Y + (long)b * ldy, nullptr, ldy, nrhs,
                      st);
  // the lower sub-block first, then the upper one through U_ab (b1 x b2)
  return diag256<T>(b2, b1, inv + (nbt + bi + 1) * iblk, LU + (long)b * lda + b + b1, lda,
                    inv + (nbt + bi) * iblk, Y + (long)(b + b1) * ldy, Y + (long)b * ldy, ldy, nrhs, st);
}

// In-place solve on Y (n x nrhs, leading dimension ldy) that already holds P B.
// With `inv` (the output of tri_inverse for this factor) the diagonal blocks
// are applied as products with their inverses, otherwise by substitution.
template <typename T>
int lu_solve_upper(int n, int nrhs, const cplx<T> *LU, long lda, cplx<T> *Y, long ldy, const cplx<T> *inv,
                   hipStream_t st) {
  int rc;
  const int nb = (n + kSolveBlock - 1) / kSolveBlock;
  for (int bi = nb - 1; bi >= 0; --bi) {
    const int b = bi * kSolveBlock;
    const int bs = std::min(kSolveBlock, n - b);
    if ((rc = diag_backward<T>(n, b, bs, nrhs, LU, lda, Y, ldy, inv, st))) return rc;
    if (b > 0)
      if ((rc = gemm_sub<T>(b, nrhs, bs, LU + b, lda, Y + (long)b * ldy, ldy, Y, ldy, st))) return rc;
  }
  return HP_OK;
}

template <typename T>
int lu_solve_permuted(int n, int nrhs, const cplx<T> *LU, long lda, cplx<T> *Y, long ldy, const cplx<T> *inv,
                      hipStream_t st) {
  int rc;
  const int nb = (n + kSolveBlock - 1) / kSolveBlock;
  for (int bi = 0; bi < nb; ++bi) {
    const int b = bi * kSolveBlock;
    const int bs = std::min(kSolveBlock, n - b);
    if ((rc = diag_forward<T>(n, b, bs, nrhs, LU, lda, Y, ldy, inv, st))) return rc;
    if (b + bs < n)
      if ((rc = gemm_sub<T>(n - b - bs, nrhs, bs, LU + (long)(b + bs) * lda + b, lda, Y + (long)b * ldy, ldy,
                            Y + (long)(b + bs) * ldy, ldy, st)))
        return rc;
  }
  return lu_solve_upper<T>(n, nrhs, LU, lda, Y, ldy, inv, st);
}

template <typename T>
int solve_inverses(int n, const cplx<T> *LU, long lda, cplx<T> *inv, hipStream_t st);
template <>
int solve_inverses<float>(int n, const cplx<float> *LU, long lda, cplx<float> *inv, hipStream_t st) {
  return tri_inverse<float>(n, LU, lda, inv, 0, (n + kInvBlock - 1) / kInvBlock, true, st);
}
template <>
int solve_inverses<double>(int, const cplx<double> *, long, cplx<double> *, hipStream_t) {
  return HP_ERR_UNSUPPORTED;
}

template <typename T>
int lu_solve(int n, int nrhs, const cplx<T> *LU, long lda, const int *perm, cplx<T> *X, long ldx, cplx<T> *tmp,
             cplx<T> *inv, hipStream_t st) {
  int rc;
  const long tot = (long)n * nrhs;
  const unsigned blocks = (unsigned)((tot + 255) / 256);
  if (inv && (rc = solve_inverses<T>(n, LU, lda, inv, st))) return rc;
  hipLaunchKernelGGL(gather_rows_kernel<T>, dim3(blocks), dim3(256), 0, st, n, nrhs, perm, X, ldx, tmp,
                     (long)nrhs);
  HP_CHECK_LAUNCH();
  if ((rc = lu_solve_permuted<T>(n, nrhs, LU, lda, tmp, nrhs, inv, st))) return rc;
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
                              cplx<double> *, cplx<double> *, hipStream_t);
template int lu_solve<float>(int, int, const cplx<float> *, long, const int *, cplx<float> *, long,
                             cplx<float> *, cplx<float> *, hipStream_t);
template int lu_solve_permuted<double>(int, int, const cplx<double> *, long, cplx<double> *, long,
                                       const cplx<double> *, hipStream_t);
template int lu_solve_permuted<float>(int, int, const cplx<float> *, long, cplx<float> *, long,
                                      const cplx<float> *, hipStream_t);
template int lu_solve_upper<float>(int, int, const cplx<float> *, long, cplx<float> *, long, const cplx<float> *,
                                   hipStream_t);

size_t factor_sync_bytes(int n) {
  const int npanels = (n + kPanelWidth - 1) / kPanelWidth;
  return sizeof(unsigned) * barrier_words(kMaxPanelGroups) * (size_t)npanels;
}
size_t factor_slot_bytes() { return slot_bytes_max() + align_up(sizeof(int) * (1 + 2 * kPlanMax), 256); }

}  // namespace hp

extern "C" int hp_set_concurrency(int factorizations) {
  if (factorizations < 1 || factorizations > 256) return HP_ERR_ARG;
  return hp::g_concurrency.exchange(factorizations);
}

// Right-hand sides, iterative refinement and R-matrix extraction.
//
// The surface right-hand sides B (Sec. 3.1, step 2) are never stored: column
// c' of B is q_i in block c' and zero elsewhere, so P B is generated straight
// from the row permutation of the factorization.
//
// Refinement (Sec. 3.2; Sec. 3.4, step 7) runs entirely on the device: the
// FP64 residual r = B - C X is formed from the block structure of C
// (Eq. block_structure) instead of an N x N FP64 matrix:
//   (C X)[(c,i)] = h sum_j TL_ij X[(c,j)] + (h l_c(l_c+1)/r_i^2 + eps_c - E) X[(c,i)]
//                  + sum_c' V_cc'(r_i) X[(c',i)],
// which costs nc nr^2 + nr nc^2 complex operations per column instead of
// (nc nr)^2.  The kinetic part is a real x complex product per channel
// (residual_local_kernel); the coupling part is one complex GEMM per radial
// point (batched MFMA gemm_sub).  A non-local system (Sec. 2: full coupling
// blocks sqrt(w_i w_j) W_cc'(r_i, r_j)) adds one FP64 GEMM with its n x n
// kernel values: T = -W (s X) with s_j = sqrt(w_j) is written into R first,
// and residual_local_kernel folds s_i T_i into the row it writes.
#include "common.h"

#include <mutex>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <vector>

namespace hp {

// P B in working precision: Y[i][c'] = B[perm[i]][c'], scaled by 1/s[c'] if s given.
template <typename T>
__global__ void rhs_from_perm_kernel(int nc, int nr, const int *__restrict__ perm, const double *__restrict__ q,
                                     cplx<T> *__restrict__ Y) {
  const long n = (long)nc * nr;
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * nc) return;
  const long i = e / nc;
  const int col = (int)(e - i * nc);
  const int src = perm[i];
  const int c = src / nr, ii = src - (src / nr) * nr;
  Y[e] = cplx<T>{(T)((c == col) ? q[ii] : 0.0), T(0)};
}

// r = B - (h TL (x) I_c) X - diag X, for a column tile of 32 and one channel;
// with w (non-local systems) R holds T = -W (s X) on entry and
// r + sqrt(w_i) T is written.
constexpr int kResCols = 32;
__global__ __launch_bounds__(256) void residual_local_kernel(int nc, int nr, double h, double E,
                                                             const double *__restrict__ tl,
                                                             const double *__restrict__ r,
                                                             const int *__restrict__ l,
                                                             const double *__restrict__ eps,
                                                             const double *__restrict__ q,
                                                             const double *__restrict__ w,
                                                             const cplx<double> *__restrict__ X,
                                                             cplx<double> *__restrict__ R) {
  extern __shared__ __align__(16) char smem_raw[];
  cplx<double> *Xs = reinterpret_cast<cplx<double> *>(smem_raw);  // [nr][kResCols]
  const int c = blockIdx.y;
  const int col0 = blockIdx.x * kResCols;
  const int ncw = min(kResCols, nc - col0);
  const int tid = threadIdx.x;
  const cplx<double> *Xc = X + (long)c * nr * nc;
  for (int e = tid; e < nr * kResCols; e += 256) {
    const int j = e / kResCols, cc = e - j * kResCols;
    Xs[e] = (cc < ncw) ? Xc[(long)j * nc + col0 + cc] : cplx<double>{0.0, 0.0};
  }
  __syncthreads();
  const int lc = l[c];
  const double shift = eps[c] - E;
  for (int e = tid; e < nr * kResCols; e += 256) {
    const int i = e / kResCols, cc = e - i * kResCols;
    if (cc >= ncw) continue;
    const double *trow = tl + (long)i * nr;
    double sr = 0.0, si = 0.0;
    for (int j = 0; j < nr; ++j) {
      const double t = trow[j];
      sr += t * Xs[j * kResCols + cc].re;
      si += t * Xs[j * kResCols + cc].im;
    }
    const double ri = r[i];
    const double dg = h * (double)lc * (double)(lc + 1) / (ri * ri) + shift;
    const cplx<double> x = Xs[i * kResCols + cc];
    const int col = col0 + cc;
    const double b = (col == c) ? q[i] : 0.0;
    cplx<double> out{b - h * sr - dg * x.re, -h * si - dg * x.im};
    const long o = ((long)c * nr + i) * nc + col;
    if (w) {
      const double si_w = sqrt(w[i]);
      const cplx<double> t = R[o];
      out.re += si_w * t.re;
      out.im += si_w * t.im;
    }
    R[o] = out;
  }
}

// Xs[(c,j)][col] = sqrt(w_j) X[(c,j)][col] (the right operand of the
// non-local residual product).
__global__ void scale_rows_sqrtw_kernel(long n, int nr, int nc, const double *__restrict__ w,
                                        const cplx<double> *__restrict__ X, cplx<double> *__restrict__ Xs) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * nc) return;
  const long row = e / nc;
  const double s = sqrt(w[row % nr]);
  const cplx<double> x = X[e];
  Xs[e] = cplx<double>{s * x.re, s * x.im};
}

// out[(c,i)] = sum over (c',j) of sqrt(w_i w_j) (|Re W| + |Im W|): the
// non-local part of the row sums of |C| (one workgroup per row).
__global__ __launch_bounds__(256) void nl_rowsum_kernel(long n, int nr, const double *__restrict__ w,
                                                        const cplx<double> *__restrict__ W, double *__restrict__ out) {
  __shared__ double part[4];
  const long row = blockIdx.x;
  const cplx<double> *wr = W + row * n;
  double sum = 0.0;
  for (long col = threadIdx.x; col < n; col += 256) {
    const cplx<double> v = wr[col];
    sum += sqrt(w[col % nr]) * (fabs(v.re) + fabs(v.im));
  }
  for (int off = 32; off > 0; off >>= 1) sum += __shfl_xor(sum, off);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = sum;
  __syncthreads();
  if (threadIdx.x == 0) out[row] = sqrt(w[row % nr]) * (part[0] + part[1] + part[2] + part[3]);
}

// Per-column max of |Re|+|Im| into out[col] (non-negative doubles compare as
// their bit patterns).  Thread (col, r0) scans rows r0, r0 + step, ...; one
// atomic per thread.  A second array, if given, is reduced into out2.
__global__ void colmax_kernel(long nrows, int ncols, const cplx<double> *__restrict__ V,
                              unsigned long long *__restrict__ out, const cplx<double> *__restrict__ V2,
                              unsigned long long *__restrict__ out2) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const int col = (int)(e % ncols);
  const long r0 = e / ncols;
  const long step = ((long)gridDim.x * blockDim.x) / ncols;
  if (step == 0 || r0 >= step) return;
  double m = 0.0, m2 = 0.0;
  for (long rr = r0; rr < nrows; rr += step) {
    const cplx<double> v = V[rr * ncols + col];
    m = fmax(m, fabs(v.re) + fabs(v.im));
    if (V2) {
      const cplx<double> w = V2[rr * ncols + col];
      m2 = fmax(m2, fabs(w.re) + fabs(w.im));
    }
  }
  atomicMax(&out[col], (unsigned long long)__double_as_longlong(m));
  if (V2) atomicMax(&out2[col], (unsigned long long)__double_as_longlong(m2));
}

__global__ void zero_u64_kernel(unsigned long long *p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0ull;
}

// Y = P r / s (working precision), s[col] = max|r_col| (1 if zero).
template <typename T>
__global__ void scale_perm_kernel(long n, int nc, const int *__restrict__ perm, const cplx<double> *__restrict__ Rr,
                                  const unsigned long long *__restrict__ smax, cplx<T> *__restrict__ Y) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * nc) return;
  const long i = e / nc;
  const int col = (int)(e - i * nc);
  double s = __longlong_as_double((long long)smax[col]);
  const double inv = (s > 0.0) ? 1.0 / s : 1.0;
  const cplx<double> v = Rr[(long)perm[i] * nc + col];
  Y[e] = cplx<T>{(T)(v.re * inv), (T)(v.im * inv)};
}

// X += s * D (FP64); per-column max |s D| into dmax (same scan order as colmax).
template <typename T>
__global__ void update_kernel(long n, int nc, const cplx<T> *__restrict__ D, const unsigned long long *__restrict__ smax,
                              cplx<double> *__restrict__ X, unsigned long long *__restrict__ dmax) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const int col = (int)(e % nc);
  const long r0 = e / nc;
  const long step = ((long)gridDim.x * blockDim.x) / nc;
  if (step == 0 || r0 >= step) return;
  const double s = __longlong_as_double((long long)smax[col]);
  const double f = (s > 0.0) ? s : 1.0;
  double m = 0.0;
  for (long rr = r0; rr < n; rr += step) {
    const long k = rr * nc + col;
    const cplx<T> d = D[k];
    const double dr = f * (double)d.re, di = f * (double)d.im;
    cplx<double> x = X[k];
    x.re += dr;
    x.im += di;
    X[k] = x;
    m = fmax(m, fabs(dr) + fabs(di));
  }
  atomicMax(&dmax[col], (unsigned long long)__double_as_longlong(m));
}

// |C|_inf (max row sum of |Re|+|Im|) from the block structure, and |B|_inf.
__global__ void cnorm_kernel(int nc, int nr, double h, double E, const double *__restrict__ tl,
                             const double *__restrict__ r, const int *__restrict__ l, const double *__restrict__ eps,
                             const double *__restrict__ v, const double *__restrict__ q,
                             const double *__restrict__ nlsum, unsigned long long *__restrict__ out) {
  const long row = (long)blockIdx.x * blockDim.x + threadIdx.x;
  double sum = 0.0, qm = 0.0;
  if (row < (long)nc * nr) {
    const int c = (int)(row / nr), i = (int)(row - (long)c * nr);
    const double *trow = tl + (long)i * nr;
    for (int j = 0; j < nr; ++j)
      if (j != i) sum += h * fabs(trow[j]);
    const int lc = l[c];
    const double dg = h * trow[i] + h * (double)lc * (lc + 1) / (r[i] * r[i]) + eps[c] - E;
    const double *vrow = v + 2 * ((long)i * nc + c) * nc;
    for (int cp = 0; cp < nc; ++cp) {
      double re = vrow[2 * cp], im = vrow[2 * cp + 1];
      if (cp == c) re += dg;
      sum += fabs(re) + fabs(im);
    }
    if (nlsum) sum += nlsum[row];
    qm = fabs(q[i]);
  }
  for (int off = 32; off > 0; off >>= 1) {
    sum = fmax(sum, __shfl_xor(sum, off));
    qm = fmax(qm, __shfl_xor(qm, off));
  }
  if ((threadIdx.x & 63) == 0) {
    atomicMax(&out[0], (unsigned long long)__double_as_longlong(sum));
    atomicMax(&out[1], (unsigned long long)__double_as_longlong(qm));
  }
}

// FP64 copy of a working-precision solution.
template <typename T>
__global__ void widen_kernel(long count, const cplx<T> *__restrict__ S, cplx<double> *__restrict__ X) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= count) return;
  const cplx<T> s = S[e];
  X[e] = cplx<double>{(double)s.re, (double)s.im};
}

static unsigned nblk(long count) { return (unsigned)((count + 255) / 256); }

// `scratch`: n x nc complex128 of free device memory (used by non-local
// systems for sqrt(w) X).
static int residual(const hp_system *sys, double E, const cplx<double> *X, cplx<double> *R, cplx<double> *scratch,
                    hipStream_t st) {
  const int nc = sys->nc, nr = sys->nr;
  const size_t shm = (size_t)nr * kResCols * sizeof(cplx<double>);
  if (shm > 150 * 1024) return HP_ERR_UNSUPPORTED;
  int rc0 = ensure_dynamic_lds((const void *)residual_local_kernel, shm);
  if (rc0) return rc0;
  dim3 grid((nc + kResCols - 1) / kResCols, nc);
  const long n = (long)nc * nr;
  if (sys->vnl) {
    const long cnt = n * nc;
    hipLaunchKernelGGL(scale_rows_sqrtw_kernel, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, st, n, nr, nc,
                       sys->w, X, scratch);
    HP_CHECK_LAUNCH();
    if ((rc0 = gemm_set_batched<double>((int)n, nc, (int)n, -1.0, (const cplx<double> *)sys->vnl, n, 0, scratch, nc,
                                        0, R, nc, 0, 1, st)))
      return rc0;
  }
  TraceScope ts(TR_RESIDUAL, st, 4.0 * (double)nc * nr * nr * nc, 0.0);
  hipLaunchKernelGGL(residual_local_kernel, grid, dim3(256), shm, st, nc, nr, sys->hbar2_2mu, E, sys->tl, sys->r,
                     sys->l, sys->eps, sys->q, sys->vnl ? sys->w : nullptr, X, R);
  HP_CHECK_LAUNCH();
  // coupling part: for every radial point i, R_i -= V_i X_i with
  // V_i = V[i] (nc x nc), X_i = rows (c', i) of X (stride nr rows).
  const long ld = (long)nr * nc;
  return gemm_sub_batched<double>(nc, nc, nc, (const cplx<double> *)sys->v, nc, (long)nc * nc, X + 0, ld,
                                  (long)nc, R, ld, (long)nc, nr, st);
}

static double u64_as_double(unsigned long long u) {
  double d;
  std::memcpy(&d, &u, sizeof(d));
  return d;
}

// Whether hp_solve replays its FP32 refinement solves from a captured graph.
std::atomic<int> g_solve_graphs{1};

// Captured refinement solves, kept across hp_solve calls.  A capture records
// kernel launches whose arguments are the factor, workspace and right-hand
// side addresses and the sizes; a later call with the same (device, n, nc,
// factor address and leading dimension, workspace address) replays the same
// launches on the memory it names, so it reuses the executable.  The first
// kSolveGraphCache keys are kept for the life of the process (never
// destroyed, so no executable is released while another thread may launch
// it, and none while the runtime shuts down at exit); a call with a key
// beyond them captures a graph of its own and releases it on return.
struct SolveGraphKey {
  int dev, n, nc;
  const void *lu;
  long lda;
  const void *work;
  bool operator==(const SolveGraphKey &o) const {
    return dev == o.dev && n == o.n && nc == o.nc && lu == o.lu && lda == o.lda && work == o.work;
  }
};
struct SolveGraphEntry {
  SolveGraphKey key;
  hipGraphExec_t exec;
};
constexpr int kSolveGraphCache = 64;
namespace {
std::mutex g_sg_mu;
SolveGraphEntry g_sg[kSolveGraphCache];
int g_sg_count = 0;
}  // namespace

static hipGraphExec_t solve_graph_find(const SolveGraphKey &key) {
  std::lock_guard<std::mutex> lk(g_sg_mu);
  for (int i = 0; i < g_sg_count; ++i)
    if (g_sg[i].key == key) return g_sg[i].exec;
  return nullptr;
}

// Keeps x for key if there is room (returns true), else the caller owns it.
static bool solve_graph_keep(const SolveGraphKey &key, hipGraphExec_t x) {
  std::lock_guard<std::mutex> lk(g_sg_mu);
  if (g_sg_count >= kSolveGraphCache) return false;
  g_sg[g_sg_count++] = SolveGraphEntry{key, x};
  return true;
}

// An executable owned by one hp_solve call (released on scope exit).
struct OwnedGraph {
  hipGraphExec_t exec = nullptr;
  OwnedGraph() = default;
  OwnedGraph(const OwnedGraph &) = delete;
  OwnedGraph &operator=(const OwnedGraph &) = delete;
  ~OwnedGraph() {
    if (exec) (void)hipGraphExecDestroy(exec);
  }
};

// Refinement loop (Sec. 3.2).  Each pass forms the FP64 residual of the
// current X, solves for the correction with the working-precision factors and
// adds it in FP64.  The size of the correction, max_c |d_c| / |x_c|, measures
// the forward error of the iterate before it; the loop stops
//  * converged when it is <= tol (tol <= 0: kRefineTol = 2^-29, after which
//    the remaining error is below the FP64 floor), or when it stops shrinking
//    (a correction larger than half the previous one: the iterate is at the
//    accuracy an FP64 residual can resolve) with the stalled correction
//    itself <= max(tol, kStallTol = 2^-26);
//  * not converged when it stops shrinking above that level (the factors are
//    too inaccurate for the refinement to contract: Performance Results,
//    Accuracy Validation, Fig. illcond) or after max_refine corrections.
// The normwise backward error max_c |r_c| / (|C| |x_c| + |b_c|) of the last
// residual is reported alongside.
//
// With `sch` (the Woodbury-kinetic form, Sec. 3.3) the factors are those of
// S = K_diag^-1 C: the right-hand sides are K^-1 q / h in every channel block
// (qt), and each residual is transformed per channel, rt_c = (kinv/h) r_c (one
// batched FP64 GEMM over the channels with the complex copy kc of kinv/h),
// before it is scaled and solved; the residual, its norm and the backward
// error stay those of C(E).
struct SchurOps {
  const cplx<double> *kc;     // nr x nr: kinv / h as complex128
  const double *qt;           // nr: kinv q / h
  cplx<double> *rt;           // n x nc: transformed residual
  unsigned long long *tmax;   // nc: its column maxima
};

template <typename T>
static int solve_impl(const hp_system *sys, double E, const cplx<T> *LU, long lda, const int *perm,
                      const int *finfo, cplx<double> *X, int max_refine, double tol, char *work,
                      const Workspace &ws, hp_solve_info *info, hipStream_t st, const SchurOps *sch = nullptr) {
  const int nc = sys->nc, nr = sys->nr;
  const long n = (long)nc * nr;
  const long cnt = n * nc;
  int rc;
  if (info) {
    info->iterations = 0;
    info->converged = 0;
    info->correction = -1.0;
    info->residual = -1.0;
  }
  cplx<T> *Y = (cplx<T> *)(work + ws.rhs_off);
  cplx<double> *Rr = (cplx<double> *)(work + ws.res_off);
  unsigned long long *smax = (unsigned long long *)(work + ws.red_off);
  unsigned long long *xmax = smax + nc;
  unsigned long long *dmax = xmax + nc;
  unsigned long long *norms = dmax + nc;  // |C|_inf, |B|_inf
  // FP32 factors: the forward substitution in the transformed form (its
  // chain is GEMMs only), built once here for all the solves of the
  // refinement; the solution lands in a second buffer (Ysol)
  cplx<T> *Ysol = Y;
  if constexpr (sizeof(T) == sizeof(float)) {
    cplx<float> *inv = (cplx<float> *)(work + ws.inv_off);
    if ((rc = solve_inverses<float>((int)n, LU, lda, inv, st))) return rc;
    if ((rc = wform_build((int)n, LU, lda, inv, (cplx<float> *)(work + ws.inv2_off), (cplx<float> *)(work + ws.wtmp_off),
                          (cplx<float> *)(work + ws.wv_off), st)))
      return rc;
    Ysol = (cplx<float> *)(work + ws.z_off);
  }
  // The refinement solves are the same ~300 launches on the same buffers each
  // time: with FP32 factors they are captured (at the first refinement solve
  // of the first call on these buffers, after the initial solve has run
  // eagerly) into a HIP graph that is replayed on the caller's stream, which
  // removes the per-launch gaps; the executable is kept for later calls.
  const bool graphs = g_solve_graphs.load(std::memory_order_relaxed) != 0;
  hipGraphExec_t sg_exec = nullptr;
  OwnedGraph owned;
  auto solve_y = [&](bool eager) -> int {
    if constexpr (sizeof(T) == sizeof(float)) {
      auto run = [&](hipStream_t s) {
        return wform_solve((int)n, nc, LU, lda, (const cplx<float> *)(work + ws.inv_off),
                           (const cplx<float> *)(work + ws.wv_off), (const cplx<float> *)(work + ws.inv2_off), Y, nc,
                           Ysol, nc, s);
      };
      if (eager || !graphs) return run(st);
      if (!sg_exec) {
        int dev = 0;
        HP_CHECK_HIP(hipGetDevice(&dev));
        const SolveGraphKey key{dev, (int)n, nc, (const void *)LU, lda, (const void *)work};
        sg_exec = solve_graph_find(key);
        if (!sg_exec) {
          hipStream_t cap = nullptr;
          HP_CHECK_HIP(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
          HP_CHECK_HIP(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal));
          const int rc1 = run(cap);
          hipGraph_t g = nullptr;
          const hipError_t e = hipStreamEndCapture(cap, &g);
          (void)hipStreamDestroy(cap);
          hipGraphExec_t x = nullptr;
          hipError_t ei = hipSuccess;
          if (!rc1 && e == hipSuccess) ei = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
          if (g) (void)hipGraphDestroy(g);  // the executable does not need it
          if (rc1) return rc1;
          HP_CHECK_HIP(e);
          HP_CHECK_HIP(ei);
          if (!solve_graph_keep(key, x)) owned.exec = x;
          sg_exec = x;
        }
      }
      HP_CHECK_HIP(hipGraphLaunch(sg_exec, st));
      return HP_OK;
    } else {
      (void)eager;
      return lu_solve_permuted<T>((int)n, nc, LU, lda, Y, nc, nullptr, st);
    }
  };
  // initial solve
  hipLaunchKernelGGL(rhs_from_perm_kernel<T>, dim3(nblk(cnt)), dim3(256), 0, st, nc, nr, perm,
                     sch ? sch->qt : sys->q, Y);
  HP_CHECK_LAUNCH();
  if ((rc = solve_y(true))) return rc;
  hipLaunchKernelGGL(widen_kernel<T>, dim3(nblk(cnt)), dim3(256), 0, st, cnt, Ysol, X);
  HP_CHECK_LAUNCH();
  int hinfo = 0;
  if (finfo) {
    HP_CHECK_HIP(hipMemcpyAsync(&hinfo, finfo, sizeof(int), hipMemcpyDeviceToHost, st));
    HP_CHECK_HIP(hipStreamSynchronize(st));
    if (hinfo == -1) return HP_ERR_SYNC;
    if (hinfo > 0) return HP_ERR_SINGULAR;
  }
  if (max_refine <= 0) {
    if (info) info->converged = 1;
    return HP_OK;
  }
  const double corr_tol = (tol > 0.0) ? tol : kRefineTol;
  const double stall_ok = std::max(corr_tol, kStallTol);
  hipLaunchKernelGGL(zero_u64_kernel, dim3(nblk(3 * nc + 2)), dim3(256), 0, st, smax, 3 * nc + 2);
  HP_CHECK_LAUNCH();
  double *nlsum = nullptr;
  if (sys->vnl) {  // Rr is free until the first residual
    nlsum = (double *)Rr;
    hipLaunchKernelGGL(nl_rowsum_kernel, dim3((unsigned)n), dim3(256), 0, st, n, nr, sys->w,
                       (const cplx<double> *)sys->vnl, nlsum);
    HP_CHECK_LAUNCH();
  }
  hipLaunchKernelGGL(cnorm_kernel, dim3(nblk(n)), dim3(256), 0, st, nc, nr, sys->hbar2_2mu, E, sys->tl, sys->r,
                     sys->l, sys->eps, sys->v, sys->q, nlsum, norms);
  HP_CHECK_LAUNCH();
  std::vector<unsigned long long> h(3 * (size_t)nc + 2);
  double corr_prev = INFINITY;
  const unsigned cm_blocks = (unsigned)std::min<long>(2048, std::max<long>(1, (n * nc + 255) / 256));
  for (int it = 0;; ++it) {
    // the working-precision right-hand sides are free until scale_perm_kernel
    if ((rc = residual(sys, E, X, Rr, (cplx<double> *)(work + ws.rhs_off), st))) return rc;
    {
      TraceScope ts(TR_REFINE, st, 0.0, 32.0 * (double)cnt);
      hipLaunchKernelGGL(zero_u64_kernel, dim3(nblk(2 * nc)), dim3(256), 0, st, smax, 2 * nc);
      HP_CHECK_LAUNCH();
      hipLaunchKernelGGL(colmax_kernel, dim3(cm_blocks), dim3(256), 0, st, n, nc, Rr, smax,
                         (const cplx<double> *)X, xmax);
      HP_CHECK_LAUNCH();
    }
    HP_CHECK_HIP(hipMemcpyAsync(h.data(), smax, (3 * nc + 2) * sizeof(unsigned long long), hipMemcpyDeviceToHost, st));
    HP_CHECK_HIP(hipStreamSynchronize(st));
    const double cn = u64_as_double(h[3 * nc]), bn = u64_as_double(h[3 * nc + 1]);
    double eta = 0.0, corr = 0.0;
    for (int c = 0; c < nc; ++c) {
      const double s = u64_as_double(h[c]), x = u64_as_double(h[nc + c]), d = u64_as_double(h[2 * nc + c]);
      eta = std::max(eta, s / (cn * x + bn));
      if (x > 0) corr = std::max(corr, d / x);
    }
    if (info) {
      info->iterations = it;
      info->residual = eta;
      if (it > 0) info->correction = corr;
    }
    if (!(eta == eta) || !(corr == corr)) return HP_ERR_NOCONV;  // NaN
    if (it > 0) {
      if (corr <= corr_tol) {
        if (info) info->converged = 1;
        return HP_OK;
      }
      if (corr > 0.5 * corr_prev) {  // stopped shrinking
        if (corr <= stall_ok) {
          if (info) info->converged = 1;
          return HP_OK;
        }
        return HP_ERR_NOCONV;
      }
      corr_prev = corr;
    }
    if (it >= max_refine) return HP_ERR_NOCONV;
    // the right-hand side of the correction solve and its column scales
    const cplx<double> *rsrc = Rr;
    const unsigned long long *rscale = smax;
    if (sch) {
      if ((rc = gemm_set_batched<double>(nr, nc, nr, 1.0, sch->kc, nr, 0, Rr, nc, (long)nr * nc, sch->rt, nc,
                                         (long)nr * nc, nc, st)))
        return rc;
      TraceScope ts(TR_REFINE, st, 0.0, 16.0 * cnt);
      hipLaunchKernelGGL(zero_u64_kernel, dim3(nblk(nc)), dim3(256), 0, st, sch->tmax, nc);
      HP_CHECK_LAUNCH();
      hipLaunchKernelGGL(colmax_kernel, dim3(cm_blocks), dim3(256), 0, st, n, nc, (const cplx<double> *)sch->rt,
                         sch->tmax, (const cplx<double> *)nullptr, (unsigned long long *)nullptr);
      HP_CHECK_LAUNCH();
      rsrc = sch->rt;
      rscale = sch->tmax;
    }
    {
      TraceScope ts(TR_REFINE, st, 0.0, 16.0 * cnt + sizeof(cplx<T>) * (double)cnt);
      hipLaunchKernelGGL(scale_perm_kernel<T>, dim3(nblk(cnt)), dim3(256), 0, st, n, nc, perm, rsrc, rscale, Y);
      HP_CHECK_LAUNCH();
    }
    if ((rc = solve_y(false))) return rc;
    {
      TraceScope ts(TR_REFINE, st, 0.0, (sizeof(cplx<T>) + 32.0) * (double)cnt);
      hipLaunchKernelGGL(zero_u64_kernel, dim3(nblk(nc)), dim3(256), 0, st, dmax, nc);
      HP_CHECK_LAUNCH();
      hipLaunchKernelGGL(update_kernel<T>, dim3(cm_blocks), dim3(256), 0, st, n, nc, Ysol, rscale, X, dmax);
      HP_CHECK_LAUNCH();
    }
  }
}

// R[c][c'] = (h/a) sum_i q_i X[(c,i)][c']
__global__ void rmatrix_kernel(int nc, int nr, double scale, const double *__restrict__ q,
                               const cplx<double> *__restrict__ X, cplx<double> *__restrict__ R) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long)nc * nc) return;
  const int c = (int)(e / nc), cp = (int)(e - (long)c * nc);
  double sr = 0.0, si = 0.0;
  for (int i = 0; i < nr; ++i) {
    const cplx<double> x = X[((long)c * nr + i) * nc + cp];
    sr += q[i] * x.re;
    si += q[i] * x.im;
  }
  R[e] = cplx<double>{scale * sr, scale * si};
}

}  // namespace hp

using namespace hp;

static bool sys_ok(const hp_system *sys) {
  return sys && sys->nc >= 1 && sys->nr >= 1 && sys->a > 0 && sys->r && sys->q && sys->tl && sys->l && sys->eps &&
         sys->v && (!sys->vnl || sys->w);
}

extern "C" int hp_solve(const hp_system *sys, double E, int prec, const void *LU, long lda, const int *perm,
                        const int *info_factor, double *X, int max_refine, double tol, void *work,
                        size_t work_bytes, hp_solve_info *info, void *stream) {
  if (!sys_ok(sys) || !LU || !perm || !X || !work) return HP_ERR_ARG;
  const long n = (long)sys->nc * sys->nr;
  if (lda < n || !prec_ok(prec) || max_refine < 0) return HP_ERR_ARG;
  Workspace ws = plan_workspace((int)n, sys->nc, prec);
  if (work_bytes < ws.total) return HP_ERR_WORKSPACE;
  hipStream_t st = (hipStream_t)stream;
  if (prec == HP_C128)
    return solve_impl<double>(sys, E, (const cplx<double> *)LU, lda, perm, info_factor, (cplx<double> *)X,
                              max_refine, tol, (char *)work, ws, info, st);
  return solve_impl<float>(sys, E, (const cplx<float> *)LU, lda, perm, info_factor, (cplx<double> *)X,
                           max_refine, tol, (char *)work, ws, info, st);
}

// Woodbury-kinetic solves: workspace = hp_solve's, then rt, kc, qt, tmax.
static size_t schur_extra_off(int n, int nrhs, int prec) { return plan_workspace(n, nrhs, prec).total; }
static size_t schur_bytes(int n, int nrhs, int prec) {
  const int nr = n / nrhs;
  return schur_extra_off(n, nrhs, prec) + align_up((size_t)n * nrhs * sizeof(cplx<double>), 256) +
         align_up((size_t)nr * nr * sizeof(cplx<double>), 256) + align_up((size_t)nr * sizeof(double), 256) +
         align_up((size_t)nrhs * sizeof(unsigned long long), 256);
}

extern "C" size_t hp_schur_workspace_bytes(int n, int nrhs, int prec) {
  if (n < 1 || nrhs < 1 || n % nrhs != 0 || !prec_ok(prec)) return 0;
  return schur_bytes(n, nrhs, prec);
}

// kc = kinv / h as complex128, qt = kinv q / h.
__global__ void schur_setup_kernel(int nr, double inv_h, const double *__restrict__ kinv, const double *__restrict__ q,
                                   cplx<double> *__restrict__ kc, double *__restrict__ qt) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e < nr * nr) kc[e] = cplx<double>{kinv[e] * inv_h, 0.0};
  if (e < nr) {
    double s = 0.0;
    for (int j = 0; j < nr; ++j) s += kinv[(long)e * nr + j] * q[j];
    qt[e] = s * inv_h;
  }
}

extern "C" int hp_solve_schur(const hp_system *sys, double E, int prec, const double *kinv, const void *LU, long lda,
                              const int *perm, const int *info_factor, double *X, int max_refine, double tol,
                              void *work, size_t work_bytes, hp_solve_info *info, void *stream) {
  if (!sys_ok(sys) || !kinv || !LU || !perm || !X || !work) return HP_ERR_ARG;
  if (sys->vnl) return HP_ERR_UNSUPPORTED;
  const long n = (long)sys->nc * sys->nr;
  if (lda < n || !prec_ok(prec) || max_refine < 0) return HP_ERR_ARG;
  if (work_bytes < schur_bytes((int)n, sys->nc, prec)) return HP_ERR_WORKSPACE;
  Workspace ws = plan_workspace((int)n, sys->nc, prec);
  hipStream_t st = (hipStream_t)stream;
  const int nr = sys->nr, nc = sys->nc;
  char *extra = (char *)work + schur_extra_off((int)n, nc, prec);
  SchurOps so;
  so.rt = (cplx<double> *)extra;
  extra += align_up((size_t)n * nc * sizeof(cplx<double>), 256);
  cplx<double> *kc = (cplx<double> *)extra;
  so.kc = kc;
  extra += align_up((size_t)nr * nr * sizeof(cplx<double>), 256);
  double *qt = (double *)extra;
  so.qt = qt;
  extra += align_up((size_t)nr * sizeof(double), 256);
  so.tmax = (unsigned long long *)extra;
  hipLaunchKernelGGL(schur_setup_kernel, dim3(nblk((long)nr * nr)), dim3(256), 0, st, nr, 1.0 / sys->hbar2_2mu, kinv,
                     sys->q, kc, qt);
  HP_CHECK_LAUNCH();
  if (prec == HP_C128)
    return solve_impl<double>(sys, E, (const cplx<double> *)LU, lda, perm, info_factor, (cplx<double> *)X,
                              max_refine, tol, (char *)work, ws, info, st, &so);
  return solve_impl<float>(sys, E, (const cplx<float> *)LU, lda, perm, info_factor, (cplx<double> *)X, max_refine,
                           tol, (char *)work, ws, info, st, &so);
}

extern "C" int hp_set_solve_graphs(int on) {
  if (on != 0 && on != 1) return HP_ERR_ARG;
  return g_solve_graphs.exchange(on);
}

extern "C" int hp_rmatrix(const hp_system *sys, const double *X, double *R, void *stream) {
  if (!sys || sys->nc < 1 || sys->nr < 1 || !(sys->a > 0) || !sys->q || !X || !R) return HP_ERR_ARG;
  const long cnt = (long)sys->nc * sys->nc;
  TraceScope ts(TR_RMATRIX, (hipStream_t)stream, 4.0 * (double)cnt * sys->nr, 16.0 * (double)cnt * sys->nr);
  hipLaunchKernelGGL(rmatrix_kernel, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, (hipStream_t)stream,
                     sys->nc, sys->nr, sys->hbar2_2mu / sys->a, sys->q, (const cplx<double> *)X,
                     (cplx<double> *)R);
  HP_CHECK_LAUNCH();
  return HP_OK;
}

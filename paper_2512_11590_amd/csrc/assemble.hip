// Matrix assembly C(E) directly in HBM (Eq. block_structure).
//
// One workgroup per matrix row (c, i); its 256 lanes sweep the row in
// contiguous 256-element strips, so every store is a fully coalesced burst.
// The kernel is bound by HBM write bandwidth: N^2 complex elements written,
// O(nr^2 + nr nc^2) bytes read (TL, V), which stay in L2.  A non-local
// system (Sec. 2: full coupling blocks) adds sqrt(w_i w_j) W_cc'(r_i, r_j)
// to every element, a second coalesced N^2 stream (its FP64 values read
// once); the sqrt(w) of the row's channel block sit in LDS.
#include "common.h"

namespace hp {

template <typename T, bool NL>
__global__ __launch_bounds__(256) void assemble_kernel(int nc, int nr, double h, double E,
                                                       const double *__restrict__ tl,
                                                       const double *__restrict__ r,
                                                       const int *__restrict__ l,
                                                       const double *__restrict__ eps,
                                                       const double *__restrict__ v,
                                                       const double *__restrict__ w,
                                                       const cplx<double> *__restrict__ vnl,
                                                       cplx<T> *__restrict__ C, long ldc) {
  extern __shared__ __align__(16) char smem_raw[];
  double *sw = reinterpret_cast<double *>(smem_raw);  // [nr]: sqrt(w_j) (non-local only)
  if constexpr (NL) {
    for (int j = threadIdx.x; j < nr; j += 256) sw[j] = sqrt(w[j]);
    __syncthreads();
  }
  const long row = blockIdx.x;
  const int c = (int)(row / nr);
  const int i = (int)(row - (long)c * nr);
  const long n = (long)nc * nr;
  const int lc = l[c];
  const double ri = r[i];
  const double diag = h * (double)lc * (double)(lc + 1) / (ri * ri) + eps[c] - E;
  const double *tl_row = tl + (size_t)i * nr;
  const double *v_row = v + 2 * ((size_t)i * nc + c) * nc;  // V[i][c][*], complex
  cplx<T> *out = C + row * ldc;
  const cplx<double> *wrow = vnl + row * n;  // read only when NL
  // (cp, j) of this lane's first column, then advanced by 256 columns per strip
  long col = threadIdx.x;
  int cp = (int)(col / nr);
  int j = (int)(col - (long)cp * nr);
  for (; col < n; col += 256) {
    double re = 0.0, im = 0.0;
    if (cp == c) {
      re = h * tl_row[j];
      if (j == i) re += diag;
    }
    if (j == i) {
      re += v_row[2 * cp];
      im += v_row[2 * cp + 1];
    }
    if constexpr (NL) {
      const double f = sw[i] * sw[j];
      const cplx<double> x = wrow[col];
      re += f * x.re;
      im += f * x.im;
    }
    out[col] = cplx<T>{(T)re, (T)im};
    j += 256;
    while (j >= nr) {
      j -= nr;
      ++cp;
    }
  }
}

}  // namespace hp

using namespace hp;

extern "C" int hp_build_matrix(const hp_system *sys, double E, int prec, void *C, long ldc,
                               void *stream) {
  if (!sys || !C || !sys->tl || !sys->r || !sys->l || !sys->eps || !sys->v) return HP_ERR_ARG;
  if (sys->nc < 1 || sys->nr < 1 || (sys->vnl && !sys->w)) return HP_ERR_ARG;
  const long n = (long)sys->nc * sys->nr;
  if (ldc < n) return HP_ERR_ARG;
  hipStream_t st = (hipStream_t)stream;
  dim3 grid((unsigned)n), block(256);
  const double elt = is_c64(prec) ? 8.0 : 16.0;
  if (!prec_ok(prec)) return HP_ERR_ARG;
  const bool nl = sys->vnl != nullptr;
  const size_t shm = nl ? (size_t)sys->nr * sizeof(double) : 0;
  TraceScope ts(TR_ASSEMBLE, st, 0.0, (elt + (nl ? 16.0 : 0.0)) * (double)n * (double)n);
  const cplx<double> *W = (const cplx<double> *)sys->vnl;
  int rc;
  auto go = [&](auto kern, auto *out) {
    if (shm > 64 * 1024 && (rc = ensure_dynamic_lds((const void *)kern, shm))) return rc;
    hipLaunchKernelGGL(kern, grid, block, shm, st, sys->nc, sys->nr, sys->hbar2_2mu, E, sys->tl, sys->r, sys->l,
                       sys->eps, sys->v, sys->w, W, out, ldc);
    HP_CHECK_LAUNCH();
    return HP_OK;
  };
  if (prec == HP_C128)
    return nl ? go(assemble_kernel<double, true>, (cplx<double> *)C)
              : go(assemble_kernel<double, false>, (cplx<double> *)C);
  return nl ? go(assemble_kernel<float, true>, (cplx<float> *)C) : go(assemble_kernel<float, false>, (cplx<float> *)C);
}

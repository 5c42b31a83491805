// Matrix assembly C(E) directly in HBM (Eq. block_structure).
//
// One workgroup per matrix row (c, i); its 256 lanes sweep the row in
// contiguous 256-element strips, so every store is a fully coalesced burst.
// The kernel is bound by HBM write bandwidth: N^2 complex elements written,
// O(nr^2 + nr nc^2) bytes read (TL, V), which stay in L2.
#include "common.h"

namespace hp {

template <typename T>
__global__ __launch_bounds__(256) void assemble_kernel(int nc, int nr, double h, double E,
                                                       const double *__restrict__ tl,
                                                       const double *__restrict__ r,
                                                       const int *__restrict__ l,
                                                       const double *__restrict__ eps,
                                                       const double *__restrict__ v,
                                                       cplx<T> *__restrict__ C, long ldc) {
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
  if (sys->nc < 1 || sys->nr < 1) return HP_ERR_ARG;
  const long n = (long)sys->nc * sys->nr;
  if (ldc < n) return HP_ERR_ARG;
  hipStream_t st = (hipStream_t)stream;
  dim3 grid((unsigned)n), block(256);
  const double elt = is_c64(prec) ? 8.0 : 16.0;
  TraceScope ts(TR_ASSEMBLE, st, 0.0, elt * (double)n * (double)n);
  if (prec == HP_C128) {
    hipLaunchKernelGGL(assemble_kernel<double>, grid, block, 0, st, sys->nc, sys->nr, sys->hbar2_2mu,
                       E, sys->tl, sys->r, sys->l, sys->eps, sys->v, (cplx<double> *)C, ldc);
  } else if (is_c64(prec)) {
    hipLaunchKernelGGL(assemble_kernel<float>, grid, block, 0, st, sys->nc, sys->nr, sys->hbar2_2mu,
                       E, sys->tl, sys->r, sys->l, sys->eps, sys->v, (cplx<float> *)C, ldc);
  } else {
    return HP_ERR_ARG;
  }
  HP_CHECK_LAUNCH();
  return HP_OK;
}
